"""FP64 reference of the primal-dual TV reconstruction -- TEST INFRASTRUCTURE ONLY.

The paper's classical baseline (Sec. 2.1) is the minimiser of

    0.5 ||A f - g||^2 + alpha TV(f)   subject to f >= 0

computed with the primal-dual hybrid gradient method of Chambolle and Pock
(the paper's reference [chambolle2011first]) and stopped when the relative
change ||f_k - f_{k-1}|| / ||f_k|| reaches 1e-4 (Sec. 2.3).  TV is the
isotropic total variation with forward differences and a zero difference
across the last row / column (Neumann boundary), unsmoothed here.

Written from the method's definition: with K = (A, grad),
F(y1, y2) = 0.5 ||y1 - g||^2 + alpha sum_ij |y2_ij|, G = indicator(f >= 0) and
theta = 1, one iteration is

    y1  <- (y1 + sigma (A fbar - g)) / (1 + sigma)          (prox of sigma F1*)
    y2  <- projection of y2 + sigma grad fbar onto {|y2_ij| <= alpha}
    f'  <- max(f - tau (A* y1 + grad* y2), 0)               (prox of tau G)
    fbar <- 2 f' - f,  f <- f'

convergent for sigma tau ||K||^2 < 1, ||K||^2 <= ||A||^2 + 8.  Operators are
passed in as callables, so the same routine runs on the oracle's PAT operator
and, in the pins, on small dense matrices.
"""
from __future__ import annotations

import numpy as np


def grad(f):
    """Forward differences (dx, dy), zero across the last column / row."""
    f = np.asarray(f, dtype=np.float64)
    dx = np.zeros_like(f)
    dy = np.zeros_like(f)
    dx[:, :-1] = f[:, 1:] - f[:, :-1]
    dy[:-1, :] = f[1:, :] - f[:-1, :]
    return dx, dy


def grad_adjoint(px, py):
    """The transpose of `grad`: (grad* p)_ij, written out term by term."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    out = np.zeros_like(px)
    # dx[i, j] = f[i, j+1] - f[i, j] for j < N-1
    out[:, :-1] -= px[:, :-1]
    out[:, 1:] += px[:, :-1]
    # dy[i, j] = f[i+1, j] - f[i, j] for i < N-1
    out[:-1, :] -= py[:-1, :]
    out[1:, :] += py[:-1, :]
    return out


def tv_iso(f):
    dx, dy = grad(f)
    return float(np.sum(np.sqrt(dx * dx + dy * dy)))


def objective(forward, f, g, alpha):
    r = forward(f) - g
    return 0.5 * float(np.sum(r * r)) + alpha * tv_iso(f)


def op_norm_sq(forward, adjoint, n, iters=100, seed=0):
    """||A||^2 by power iteration on A* A (FP64)."""
    x = np.random.default_rng(seed).random((n, n))
    lam = 0.0
    for _ in range(iters):
        x = x / np.linalg.norm(x)
        y = adjoint(forward(x))
        lam = float(np.sum(x * y))
        x = y
    return lam


def step_sizes(a_norm_sq, safety=0.99):
    """sigma = tau = safety / ||K|| with ||K||^2 <= ||A||^2 + 8."""
    s = safety / np.sqrt(a_norm_sq + 8.0)
    return s, s


def pdhg(forward, adjoint, g, n, alpha, sigma, tau, iters, f0=None, tol=None, return_dual=False):
    """Run `iters` iterations (or stop early once the relative change is <= tol).
    Returns (f, history of relative changes) [+ (y1, y2x, y2y) with return_dual]."""
    g = np.asarray(g, dtype=np.float64)
    f = np.zeros((n, n)) if f0 is None else np.array(f0, dtype=np.float64)
    fbar = f.copy()
    y1 = np.zeros_like(g)
    y2x = np.zeros((n, n))
    y2y = np.zeros((n, n))
    hist = []
    for _ in range(iters):
        y1 = (y1 + sigma * (forward(fbar) - g)) / (1.0 + sigma)
        dx, dy = grad(fbar)
        vx, vy = y2x + sigma * dx, y2y + sigma * dy
        scale = np.maximum(1.0, np.sqrt(vx * vx + vy * vy) / alpha) if alpha > 0 else None
        if alpha > 0:
            y2x, y2y = vx / scale, vy / scale
        else:
            y2x, y2y = np.zeros_like(vx), np.zeros_like(vy)
        fn = np.maximum(f - tau * (adjoint(y1) + grad_adjoint(y2x, y2y)), 0.0)
        nrm = np.linalg.norm(fn)
        hist.append(float(np.linalg.norm(fn - f) / nrm) if nrm > 0 else 0.0)
        fbar = 2.0 * fn - f
        f = fn
        if tol is not None and hist[-1] <= tol:
            break
    if return_dual:
        return f, hist, (y1, y2x, y2y)
    return f, hist
