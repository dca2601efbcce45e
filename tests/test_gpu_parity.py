"""GPU parity: the HIP operator pair against the FP64 oracle (element by element).

Tolerance: relative L2 error <= 1e-5 in FP32 (the accuracy the operator is
specified to), on seeded synthetic inputs at sizes that span several tiles of
every kernel and have ragged tails (odd N/D/T, non-power-of-two FFT lengths,
arcs that are not a divisor of the circle).
"""
import math

import numpy as np
import pytest

from pat_inputs import CONFIGS, Geometry, config_geometry, make_phantom

pytestmark = pytest.mark.gpu

TOL = 1e-5

GEOMS = {
    "gradcheck": config_geometry("gradcheck"),
    "cfg1": config_geometry(1),
    # ragged: every size off the power-of-two grid, R != 1, rho_s < 1, c != 1, arc off-centre
    "ragged": Geometry(n=40, n_det=37, n_t=75, dt=2.2 / 75, arc_span=math.radians(250), arc_center=0.3,
                       c=1.3, support_r=0.95, det_r=1.1),
    # no endpoint term, higher lambda oversampling, narrow arc
    "noem": Geometry(n=48, n_det=40, n_t=96, dt=2 / 96, arc_span=math.radians(90), em_correction=0,
                     lambda_oversample=3.0),
    "cfg2": config_geometry(2),
    "cfg3": config_geometry(3),
    # 270 degrees: every third point of a 4D-point angular grid (even grid, stride 3), off-centre
    "stride3": Geometry(n=48, n_det=64, n_t=96, dt=2 / 96, arc_span=math.radians(270), arc_center=0.7),
    # 12 detectors spaced 2 pi 2/27: odd grid of 27 points, stride 2
    "stride2_odd": Geometry(n=32, n_det=12, n_t=64, dt=2 / 64, arc_span=2 * math.pi * 24 / 27),
}


def _phantom(name, geom, seed):
    if name.startswith("cfg") and name[3:].isdigit():
        nb, nd, nl = CONFIGS[int(name[3:])]["phantom"]
    else:
        nb, nd, nl = 5, 1, 1
    return make_phantom(geom.n, nb, nd, nl, seed)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_cache = {}


def _case(name):
    """(geom, f, d, A f, A* d) with the oracle results cached per module."""
    if name not in _cache:
        import oracle
        geom = GEOMS[name]
        f = _phantom(name, geom, 100 + len(_cache))
        rng = np.random.default_rng(200 + len(_cache))
        d = rng.standard_normal((geom.n_det, geom.n_t))
        _cache[name] = (geom, f, d, oracle.forward(geom, f), oracle.adjoint(geom, d))
    return _cache[name]


@pytest.mark.parametrize("name", list(GEOMS))
def test_forward_adjoint_match_oracle(torch_dev, name):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom, f, d, Af, Ad = _case(name)
    plan = pat.PatPlan(geom, max_batch=1)
    g = plan.forward(torch.tensor(f, dtype=torch.float32, device="cuda")).cpu().double().numpy()
    a = plan.adjoint(torch.tensor(d, dtype=torch.float32, device="cuda")).cpu().double().numpy()
    ef, ea = _rel(g, Af), _rel(a, Ad)
    print("%s: forward rel L2 %.3e  adjoint rel L2 %.3e" % (name, ef, ea))
    assert ef <= TOL and ea <= TOL
    # outside the support the adjoint is exactly zero
    X = -1 + (np.arange(geom.n) + 0.5) * geom.h
    outside = (X[None, :] ** 2 + X[:, None] ** 2) >= geom.support_r ** 2
    assert np.all(a[outside] == 0.0)
    plan.close()


@pytest.mark.parametrize("name", ["gradcheck", "ragged", "cfg2"])
def test_dot_product_identity(torch_dev, name):
    """<A f, d> = <f, A* d> for the GPU pair itself (FP32 rounding only)."""
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom, f, d, _, _ = _case(name)
    plan = pat.PatPlan(geom)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    dt = torch.tensor(d, dtype=torch.float32, device="cuda")
    g = plan.forward(ft).double()
    a = plan.adjoint(dt).double()
    lhs = float((g * dt.double()).sum())
    rhs = float((ft.double() * a).sum())
    err = abs(lhs - rhs) / (float(g.norm()) * float(dt.double().norm()))
    print("%s: dot identity %.3e" % (name, err))
    assert err <= TOL
    plan.close()


def test_bitwise_repeatable_and_zero(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom, f, d, _, _ = _case("ragged")
    plan = pat.PatPlan(geom)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    dt = torch.tensor(d, dtype=torch.float32, device="cuda")
    g1, g2 = plan.forward(ft).clone(), plan.forward(ft).clone()
    a1, a2 = plan.adjoint(dt).clone(), plan.adjoint(dt).clone()
    assert torch.equal(g1, g2) and torch.equal(a1, a2)
    z = plan.forward(torch.zeros_like(ft))
    za = plan.adjoint(torch.zeros_like(dt))
    assert float(z.abs().max()) == 0.0 and float(za.abs().max()) == 0.0
    plan.close()


def test_batch_equals_single(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = GEOMS["ragged"]
    B = 5
    fs = np.stack([make_phantom(geom.n, 4, 1, 1, 300 + b) for b in range(B)])
    rng = np.random.default_rng(301)
    ds = rng.standard_normal((B, geom.n_det, geom.n_t))
    plan = pat.PatPlan(geom, max_batch=B)
    ft = torch.tensor(fs, dtype=torch.float32, device="cuda")
    dt = torch.tensor(ds, dtype=torch.float32, device="cuda")
    gb, ab = plan.forward(ft).clone(), plan.adjoint(dt).clone()
    for b in range(B):
        assert torch.equal(gb[b], plan.forward(ft[b].contiguous()))
        assert torch.equal(ab[b], plan.adjoint(dt[b].contiguous()))
    plan.close()


def test_python_layer_rejects_bad_tensors(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = GEOMS["gradcheck"]
    plan = pat.PatPlan(geom, max_batch=2)
    with pytest.raises(TypeError):
        plan.forward(torch.zeros((geom.n, geom.n), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((geom.n, geom.n), dtype=torch.float32))  # CPU tensor
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((geom.n, geom.n + 1), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((geom.n, 2 * geom.n), dtype=torch.float32, device="cuda")[:, ::2])
    with pytest.raises(pat.PatError):
        plan.forward(torch.zeros((3, geom.n, geom.n), dtype=torch.float32, device="cuda"))  # batch > capacity
    plan.close()
