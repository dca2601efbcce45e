"""Pins of the FP64 primal-dual TV reference (oracle/pdhg.py), CPU only.

* grad and grad_adjoint are transposes (<grad f, p> = <f, grad* p> to 1e-12).
* alpha = 0: the iteration solves non-negative least squares; its limit equals
  scipy.optimize.nnls on a small dense problem.
* alpha > 0: its limit matches an independent solver -- L-BFGS-B with bounds
  f >= 0 on the same objective with the TV smoothed by eps = 1e-9 -- in
  objective value and in f.
* the dual TV variable stays in {|y2_ij| <= alpha} and is active; the data
  dual approaches the residual A f - g; the stopping rule of the paper
  (relative change <= 1e-4) is reached and returned.
"""
import numpy as np
import pytest
from scipy import optimize

from oracle import pdhg as pd


def _dense(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n * n)) / np.sqrt(m)
    return A, (lambda x: A @ x.ravel()), (lambda y: (A.T @ y).reshape(n, n))


def test_grad_adjoint_is_the_transpose():
    rng = np.random.default_rng(1)
    for n in (2, 5, 9):
        f = rng.standard_normal((n, n))
        px, py = rng.standard_normal((n, n)), rng.standard_normal((n, n))
        dx, dy = pd.grad(f)
        lhs = float(np.sum(dx * px) + np.sum(dy * py))
        rhs = float(np.sum(f * pd.grad_adjoint(px, py)))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # constant images have zero gradient, so grad* p sums to zero
    assert abs(float(np.sum(pd.grad_adjoint(px, py)))) < 1e-12


def test_alpha_zero_is_nonnegative_least_squares():
    n, m = 5, 60
    A, fwd, adj = _dense(m, n, 2)
    x_true = np.maximum(np.random.default_rng(3).standard_normal(n * n), 0.0)
    g = A @ x_true + 0.3 * np.random.default_rng(4).standard_normal(m)
    ref, _ = optimize.nnls(A, g)
    s, t = pd.step_sizes(pd.op_norm_sq(fwd, adj, n))
    f, hist = pd.pdhg(fwd, adj, g, n, 0.0, s, t, 20000, tol=1e-13)
    err = np.linalg.norm(f.ravel() - ref) / np.linalg.norm(ref)
    assert err < 1e-7, err


def test_tv_limit_matches_lbfgsb():
    n, m, alpha, eps = 6, 50, 0.05, 1e-9
    A, fwd, adj = _dense(m, n, 5)
    x_true = np.zeros((n, n))
    x_true[1:4, 2:5] = 1.0
    g = A @ x_true.ravel() + 0.05 * np.random.default_rng(6).standard_normal(m)

    def obj(x):
        f = x.reshape(n, n)
        r = A @ x - g
        dx, dy = pd.grad(f)
        s = np.sqrt(dx * dx + dy * dy + eps * eps)
        val = 0.5 * r @ r + alpha * s.sum()
        gr = A.T @ r + alpha * pd.grad_adjoint(dx / s, dy / s).ravel()
        return val, gr

    res = optimize.minimize(obj, np.full(n * n, 0.5), jac=True, method="L-BFGS-B",
                            bounds=[(0.0, None)] * (n * n), options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    s, t = pd.step_sizes(pd.op_norm_sq(fwd, adj, n))
    f, hist = pd.pdhg(fwd, adj, g, n, alpha, s, t, 30000, tol=1e-12)
    p_pd = pd.objective(fwd, f, g, alpha)
    p_lb = pd.objective(fwd, res.x.reshape(n, n), g, alpha)
    assert p_pd <= p_lb * (1 + 1e-6) + 1e-12          # PDHG is at least as good as the smoothed solve
    assert abs(p_pd - p_lb) <= 1e-5 * abs(p_lb)
    assert np.linalg.norm(f.ravel() - res.x) / np.linalg.norm(res.x) < 1e-2


def test_dual_projection_and_stopping_rule():
    n, m = 6, 40
    A, fwd, adj = _dense(m, n, 7)
    g = np.random.default_rng(8).standard_normal(m)
    s, t = pd.step_sizes(pd.op_norm_sq(fwd, adj, n))
    f, hist, (y1, y2x, y2y) = pd.pdhg(fwd, adj, g, n, 0.1, s, t, 5000, tol=1e-4, return_dual=True)
    assert hist[-1] <= 1e-4 and all(h > 1e-4 for h in hist[:-1])
    assert np.all(f >= 0.0)
    mag = np.sqrt(y2x ** 2 + y2y ** 2)
    assert np.all(mag <= 0.1 * (1 + 1e-12)) and mag.max() > 0.05   # feasible and active
    # at a fixed point, y1 = A f - g (the data dual is the residual)
    assert np.linalg.norm(y1 - (fwd(f) - g)) <= 1e-2 * np.linalg.norm(y1)


@pytest.mark.parametrize("cfg", ["gradcheck"])
def test_pdhg_on_the_pat_operator_decreases_the_objective(oracle_mod, cfg):
    import oracle
    from pat_inputs import config_geometry, make_phantom
    geom = config_geometry(cfg)
    fwd = lambda x: oracle.forward(geom, x)
    adj = lambda y: oracle.adjoint(geom, y)
    g = fwd(make_phantom(geom.n, 5, 1, 0, 11))
    s, t = pd.step_sizes(pd.op_norm_sq(fwd, adj, geom.n, iters=30))
    f10, _ = pd.pdhg(fwd, adj, g, geom.n, 1e-3, s, t, 10)
    f60, _ = pd.pdhg(fwd, adj, g, geom.n, 1e-3, s, t, 60)
    o0 = pd.objective(fwd, np.zeros((geom.n, geom.n)), g, 1e-3)
    assert pd.objective(fwd, f60, g, 1e-3) < pd.objective(fwd, f10, g, 1e-3) < o0
