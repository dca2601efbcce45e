"""Closed forms that pin the oracle -- TEST INFRASTRUCTURE ONLY.

None of these reuse the oracle's code path; they evaluate the same quantities
through different mathematics (special functions, continuum solutions of
eq. (1)) so that a wrong sign, index, weight or transposition in the oracle's
direct sums shows up as a mismatch.

* `discrete_gaussian_data`: for f a sum of Gaussians a exp(-|x-c|^2/(2 s^2))
  that are well resolved (s >= 3h) and well inside the support, the pixel
  Fourier transform equals 2 pi s^2 a exp(-s^2 lam^2/2) exp(-i xi.c) to
  ~1e-16, and the uniform-angle average of exp(i lam omega.(x_d - c)) equals
  J_0(lam |x_d - c|) (the Npsi-point rule is exact for that bandwidth), so
      g(d, j) = sum_n W_n cos(c lam_n t_j) sum_b 2 pi s_b^2 a_b e^{-s_b^2 lam_n^2/2} J_0(lam_n |x_d - c_b|) + kappa M0.
* `discrete_impulse_adjoint`: A* of the unit datum at (d, j) is
      h^2 m(x) [ sum_n W_n cos(c lam_n t_j) J_0(lam_n |x - x_d|) + kappa ].
* `hankel_gaussian`: the continuum solution of eq. (1)-(2) for a Gaussian,
      p(x_d, t) = a s^2 int_0^inf lam e^{-s^2 lam^2/2} J_0(lam rho) cos(c lam t) dlam.
* `poisson_gaussian`: the same solution from the 2D Poisson formula,
      p = d/dt [ t int_0^{pi/2} sin(al) Mbar(c t sin(al)) d al ],
  with Mbar(r) = a e^{-(rho^2+r^2)/(2 s^2)} I_0(rho r / s^2) the circular mean
  of the Gaussian on the circle of radius r about x_d.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def _lam_W(sz):
    n = np.arange(1, sz["n_lam"] + 1, dtype=np.float64)
    lam = n * sz["dlam"]
    return lam, lam * sz["dlam"] / (2 * math.pi)


def detector_xy(geom):
    th = np.asarray(geom.det_angles())
    return geom.det_r * np.cos(th), geom.det_r * np.sin(th)


def discrete_gaussian_data(geom, sz, blobs, mass=None):
    """Closed form of the discrete operator for a Gaussian-blob image, (D, T)."""
    lam, W = _lam_W(sz)
    xd, yd = detector_xy(geom)
    t = np.asarray(geom.times())
    S = np.zeros((geom.n_det, lam.size))  # sum over blobs of the radial spectrum times J_0
    for b in blobs:
        rho = np.hypot(xd[:, None] - b.cx, yd[:, None] - b.cy)
        S += 2 * math.pi * b.sigma ** 2 * b.amp * np.exp(-(b.sigma * lam) ** 2 / 2) * special.j0(lam * rho)
    C = np.cos(geom.c * np.outer(lam, t))  # (n_lam, T)
    if mass is None:
        mass = sum(2 * math.pi * b.sigma ** 2 * b.amp for b in blobs)
    return (S * W) @ C + sz["kappa"] * mass


def discrete_impulse_adjoint(geom, sz, d, j, flat_idx=None):
    """A* applied to the unit datum at detector d, time index j (0-based): the
    (N, N) image, or its values at the pixels with flat index i*N + j."""
    from pat_inputs import pixel_centres
    lam, W = _lam_W(sz)
    X, Y = pixel_centres(geom.n)
    if flat_idx is not None:
        X, Y = X.ravel()[flat_idx], Y.ravel()[flat_idx]
    xd, yd = detector_xy(geom)
    t = geom.times()[j]
    rho = np.hypot(X - xd[d], Y - yd[d])
    coef = W * np.cos(geom.c * lam * t)
    acc = np.zeros_like(X)
    for cn, ln in zip(coef, lam):
        acc += cn * special.j0(ln * rho)
    m = (X * X + Y * Y < geom.support_r ** 2)
    h = geom.h
    return np.where(m, h * h * (acc + sz["kappa"]), 0.0)


def _gl_composite(a, b, panels, order=20):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(a, b, panels + 1)
    mid = 0.5 * (edges[1:] + edges[:-1])
    half = 0.5 * (edges[1:] - edges[:-1])
    nodes = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    weights = (half[:, None] * w[None, :]).ravel()
    return nodes, weights


def hankel_gaussian(blob, xd, yd, t, c=1.0):
    """Continuum pressure at (xd, yd), time t, for one Gaussian blob."""
    s, a = blob.sigma, blob.amp
    rho = math.hypot(xd - blob.cx, yd - blob.cy)
    lmax = 12.0 / s
    nodes, w = _gl_composite(0.0, lmax, 4000)
    val = nodes * np.exp(-(s * nodes) ** 2 / 2) * special.j0(nodes * rho) * np.cos(c * nodes * t)
    return a * s * s * float(np.dot(w, val))


def poisson_gaussian(blob, xd, yd, t, c=1.0):
    """Same pressure from the 2D Poisson formula (an independent route)."""
    s, a = blob.sigma, blob.amp
    rho = math.hypot(xd - blob.cx, yd - blob.cy)
    al, w = _gl_composite(0.0, math.pi / 2, 4000)
    r = c * t * np.sin(al)
    z = rho * r / (s * s)
    env = a * np.exp(-((rho - r) ** 2) / (2 * s * s))  # e^{-(rho^2+r^2)/2s^2} I_0(z) = env * i0e(z)
    Mbar = env * special.i0e(z)
    dMbar = env * (-(r / (s * s)) * special.i0e(z) + (rho / (s * s)) * special.i1e(z))
    phi = float(np.dot(w, np.sin(al) * Mbar))
    dphi = float(np.dot(w, np.sin(al) * dMbar * c * np.sin(al)))
    return phi + t * dphi
