"""FP64 reference for the smoothed total variation of eq. (4)/(5) -- TEST INFRASTRUCTURE ONLY.

TV_eps(f) = sum_{i,j} sqrt(dx_ij^2 + dy_ij^2 + eps^2) with forward differences
dx_ij = f[i, j+1] - f[i, j], dy_ij = f[i+1, j] - f[i, j], and a zero
difference across the last column / row (Neumann boundary).  Its gradient is
the plain derivative of that sum.  Also: the projected-gradient objective
0.5 ||A f - g||^2 + lam TV_eps(f) of eq. (4) (constraint f >= 0).
"""
from __future__ import annotations

import numpy as np


def tv_value(f, eps):
    f = np.asarray(f, dtype=np.float64)
    dx = np.zeros_like(f)
    dy = np.zeros_like(f)
    dx[:, :-1] = f[:, 1:] - f[:, :-1]
    dy[:-1, :] = f[1:, :] - f[:-1, :]
    return float(np.sum(np.sqrt(dx * dx + dy * dy + eps * eps)))


def tv_grad(f, eps):
    f = np.asarray(f, dtype=np.float64)
    dx = np.zeros_like(f)
    dy = np.zeros_like(f)
    dx[:, :-1] = f[:, 1:] - f[:, :-1]
    dy[:-1, :] = f[1:, :] - f[:-1, :]
    s = np.sqrt(dx * dx + dy * dy + eps * eps)
    px, py = dx / s, dy / s
    g = -(px + py)
    g[:, 1:] += px[:, :-1]   # term (i, j-1) contains +f[i, j]
    g[1:, :] += py[:-1, :]   # term (i-1, j) contains +f[i, j]
    return g


def objective(geom, f, g_meas, lam, eps, forward):
    r = forward(geom, f) - g_meas
    return 0.5 * float(np.sum(r * r)) + lam * tv_value(f, eps)
