"""Pins of the FP64 TV reference and of the operator's gradient (CPU only).

The TV reference (oracle/tv.py) is checked against central finite
differences, against the closed forms of a constant image (value N^2 eps,
zero gradient) and of a linear ramp (zero gradient in the interior), and the
oracle operator's transpose is checked with torch.autograd.gradcheck (FP64)
through an oracle-backed autograd Function at the gradient-check shape
(32^2, 32 detectors on 120 deg, 64 samples).
"""
import math

import numpy as np
import pytest
import torch

from oracle import tv as tvref
from pat_inputs import config_geometry


def test_tv_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((12, 12))
    eps = 0.05
    g = tvref.tv_grad(f, eps)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 7), (11, 11), (11, 0), (5, 11), (0, 6)]:
        fp, fm = f.copy(), f.copy()
        fp[i, j] += h
        fm[i, j] -= h
        fd = (tvref.tv_value(fp, eps) - tvref.tv_value(fm, eps)) / (2 * h)
        assert abs(fd - g[i, j]) < 1e-7 * max(1.0, abs(fd))


def test_tv_constant_and_ramp():
    eps = 1e-3
    n = 16
    c = np.full((n, n), 2.5)
    assert tvref.tv_value(c, eps) == pytest.approx(n * n * eps, rel=1e-12)
    assert np.abs(tvref.tv_grad(c, eps)).max() == 0.0
    jj, ii = np.meshgrid(np.arange(n), np.arange(n))
    ramp = 0.3 * jj - 0.2 * ii
    g = tvref.tv_grad(ramp, eps)
    assert np.abs(g[1:-1, 1:-1]).max() < 1e-12     # interior: the flux is constant
    assert np.abs(g).max() > 0.1                   # boundary terms are not


class _OracleA(torch.autograd.Function):
    """A with the FP64 oracle (forward) and its transpose (backward)."""

    @staticmethod
    def forward(ctx, f, geom):
        import oracle
        ctx.geom = geom
        return torch.from_numpy(oracle.forward(geom, f.detach().numpy()))

    @staticmethod
    def backward(ctx, gout):
        import oracle
        return torch.from_numpy(oracle.adjoint(ctx.geom, gout.detach().contiguous().numpy())), None


def test_gradcheck_oracle_operator(oracle_mod):
    geom = config_geometry("gradcheck")
    rng = np.random.default_rng(6)
    f = torch.tensor(rng.standard_normal((geom.n, geom.n)), dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: _OracleA.apply(x, geom), (f,), eps=1e-6, atol=1e-7,
                                    rtol=1e-5, fast_mode=True)


def test_gradcheck_tv_objective(oracle_mod):
    """Gradient of 0.5||A f - g||^2 + lam TV_eps(f) (oracle A, reference TV) by gradcheck."""
    geom = config_geometry("gradcheck")
    rng = np.random.default_rng(7)
    g = torch.tensor(rng.standard_normal((geom.n_det, geom.n_t)), dtype=torch.float64)
    lam, eps = 1e-3, 1e-3

    class _TV(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f):
            ctx.save_for_backward(f)
            return torch.tensor(tvref.tv_value(f.detach().numpy(), eps), dtype=torch.float64)

        @staticmethod
        def backward(ctx, go):
            (f,) = ctx.saved_tensors
            return go * torch.from_numpy(tvref.tv_grad(f.detach().numpy(), eps))

    def obj(x):
        r = _OracleA.apply(x, geom) - g
        return 0.5 * (r * r).sum() + lam * _TV.apply(x)

    f = torch.tensor(rng.uniform(0, 1, (geom.n, geom.n)), dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(obj, (f,), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)
