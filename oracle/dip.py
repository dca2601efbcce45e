"""FP64 objective of the deep image prior, eq. (5) -- TEST INFRASTRUCTURE ONLY.

For the network output f (an N x N image) the objective and its gradient are

    J(f)      = ||A f - g||^2 + lam TV_eps(f)
    grad J(f) = 2 A* (A f - g) + lam grad TV_eps(f)

with the oracle's direct-sum A, A* and the smoothed isotropic TV of
oracle.tv.  The gradient in the network parameters is this image gradient
pulled back through the network (autograd), so these two functions are what a
parity check of a DIP step needs from the physics side.
"""
from __future__ import annotations

import numpy as np

from . import adjoint, forward
from .tv import tv_grad, tv_value


def objective(geom, f, g_meas, lam, eps):
    r = forward(geom, f) - np.asarray(g_meas, dtype=np.float64)
    return float(np.sum(r * r)) + lam * tv_value(f, eps)


def gradient(geom, f, g_meas, lam, eps):
    r = forward(geom, f) - np.asarray(g_meas, dtype=np.float64)
    return 2.0 * adjoint(geom, r) + lam * tv_grad(f, eps)
