"""Pins of the FP64 CGLS reference (oracle/cgls.py), CPU only.

* After rank(A) steps on a small full-rank dense problem, CGLS equals the
  least-squares solution of numpy.linalg.lstsq (1e-9).
* Every iterate equals scipy's LSQR iterate with the same number of steps
  (the two are the same Krylov method in exact arithmetic; 1e-8).
* The residual norm never increases, and A* r_k is orthogonal to A* r_j.
* On the PAT operator the data misfit falls monotonically.
"""
import numpy as np
from scipy.sparse.linalg import lsqr

from oracle.cgls import cgls


def _dense(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    return A, (lambda x: A @ x), (lambda y: A.T @ y)


def test_cgls_reaches_least_squares():
    A, fwd, adj = _dense(40, 12, 1)
    g = np.random.default_rng(2).standard_normal(40)
    f = cgls(fwd, adj, g, (12,), 12)
    ref = np.linalg.lstsq(A, g, rcond=None)[0]
    assert np.linalg.norm(f - ref) <= 1e-9 * np.linalg.norm(ref)


def test_cgls_iterates_equal_lsqr():
    A, fwd, adj = _dense(60, 25, 3)
    g = np.random.default_rng(4).standard_normal(60)
    for k in (1, 2, 5, 9):
        f = cgls(fwd, adj, g, (25,), k)
        ref = lsqr(A, g, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert np.linalg.norm(f - ref) <= 1e-8 * np.linalg.norm(ref), k


def test_residual_monotone_and_gradients_orthogonal():
    A, fwd, adj = _dense(50, 30, 5)
    g = np.random.default_rng(6).standard_normal(50)
    _, hist = cgls(fwd, adj, g, (30,), 15, return_history=True)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    f3 = cgls(fwd, adj, g, (30,), 3)
    f6 = cgls(fwd, adj, g, (30,), 6)
    s3, s6 = adj(g - fwd(f3)), adj(g - fwd(f6))
    assert abs(float(s3 @ s6)) <= 1e-9 * np.linalg.norm(s3) * np.linalg.norm(s6)


def test_cgls_on_the_pat_operator(oracle_mod):
    import oracle
    from pat_inputs import config_geometry, make_phantom
    geom = config_geometry("gradcheck")
    g = oracle.forward(geom, make_phantom(geom.n, 5, 1, 0, 12))
    fwd = lambda x: oracle.forward(geom, x)
    adj = lambda y: oracle.adjoint(geom, y)
    _, hist = cgls(fwd, adj, g, (geom.n, geom.n), 8, return_history=True)
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.2 * hist[0]
