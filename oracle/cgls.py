"""FP64 reference of CGLS, the iterative stand-in for the fast inverse -- TEST
INFRASTRUCTURE ONLY.

The network input of the paper's deep image prior (Sec. 2.2) is an approximate
inverse of the data, obtained there with a fast inversion formula from the
cited literature that the paper does not state.  The stand-in here is a few
steps of conjugate gradients on the normal equations A* A f = A* g (CGLS, the
least-squares form of Hestenes and Stiefel), started from f_0:

    r = g - A f_0,  s = A* r,  p = s,  gamma = <s, s>
    per step:  q = A p,  alpha = gamma / <q, q>
               f <- f + alpha p,  r <- r - alpha q
               s = A* r,  gamma' = <s, s>,  p <- s + (gamma' / gamma) p,  gamma <- gamma'

Step k minimises ||A f - g|| over f_0 + the Krylov space of A*A of dimension
k.  Operators are callables, so the routine runs on the oracle's PAT operator
and, in the pins, on small dense matrices.
"""
from __future__ import annotations

import numpy as np


def cgls(forward, adjoint, g, shape, iters, f0=None, return_history=False):
    """`iters` CGLS steps; returns f (and the residual norms ||g - A f_k||, k = 0..iters)."""
    g = np.asarray(g, dtype=np.float64)
    f = np.zeros(shape) if f0 is None else np.array(f0, dtype=np.float64)
    r = g - forward(f)
    s = adjoint(r)
    p = s.copy()
    gamma = float(np.sum(s * s))
    hist = [float(np.linalg.norm(r))]
    for _ in range(iters):
        if gamma == 0.0:
            hist.append(hist[-1])
            continue
        q = forward(p)
        alpha = gamma / float(np.sum(q * q))
        f = f + alpha * p
        r = r - alpha * q
        s = adjoint(r)
        gamma_new = float(np.sum(s * s))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        hist.append(float(np.linalg.norm(r)))
    if return_history:
        return f, hist
    return f
