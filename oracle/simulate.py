"""FP64 reference of the FFT wave-propagation data simulator -- TEST
INFRASTRUCTURE ONLY.

The paper's simulation study (Sec. 2.4.1, "Simulations") generates its data on a
finer Cartesian grid (512 x 512) with an FFT-based wave propagation method in
the manner of k-Wave, so that the data do not come from the reconstruction's
own discretisation (no inverse crime).  The paper gives no formulas; the
reading used here, for a constant speed of sound c:

* the fine image f (N_s x N_s pixels, cell centres on [-1, 1]^2, h_s = 2 / N_s),
  restricted to the support disc |x| < rho_s, is zero-padded to a periodic
  box of M x M cells of the same size, centred;
* the box is wide enough that no wave wraps around: its half-width
  L = M h_s / 2 satisfies 2 L - R - rho_s > c t_T (the nearest periodic copy
  of the source cannot reach a detector by the last time sample t_T) and
  L > R + 3 h_s; M is the smallest even 2^a 3^b with M - N_s even that
  meets both;
* the pressure is the exact solution of the periodic wave equation with
  p(x, 0) = f, p_t(x, 0) = 0:  p(t) = IFFT2[ FFT2(f) cos(c |k| t) ], with
  k the wave vectors 2 pi m / (M h_s) of the box (the k-space propagator,
  which is what a k-space pseudospectral scheme computes for constant c);
* the data are p(x_d, t_j) at the detectors x_d = R (cos theta_d, sin theta_d)
  and times t_j = j dt (j = 1..T), by separable Keys cubic convolution
  (a = -1/2) on the box's cell centres.
"""
from __future__ import annotations

import numpy as np


def smooth_2a3b(m: int) -> int:
    """Smallest 2^a 3^b >= m."""
    best = None
    p2 = 1
    while p2 < 2 * m + 2:
        p = p2
        while p < 2 * m + 2:
            if p >= m and (best is None or p < best):
                best = p
            p *= 3
        p2 *= 2
    return best


def box_side(ns: int, det_r: float, support_r: float, c: float, t_last: float) -> int:
    """Side M of the periodic box (cells of h_s = 2 / ns) per the rule above."""
    h = 2.0 / ns
    half = max((det_r + support_r + c * t_last) / 2.0, det_r + 3.0 * h) + h
    m = max(int(np.ceil(2.0 * half / h)), ns)
    while True:
        m = smooth_2a3b(m)
        if m % 2 == 0 and (m - ns) % 2 == 0:
            return m
        m += 1


def keys_weights(frac: float) -> np.ndarray:
    """Keys cubic convolution weights (a = -1/2) of the samples at offsets -1, 0, 1, 2."""
    a = -0.5
    s = np.array([1.0 + frac, frac, 1.0 - frac, 2.0 - frac])
    w = np.where(s <= 1.0, (a + 2) * s ** 3 - (a + 3) * s ** 2 + 1.0,
                 a * s ** 3 - 5 * a * s ** 2 + 8 * a * s - 4 * a)
    return w


def sample(field: np.ndarray, h: float, pts) -> np.ndarray:
    """Keys cubic interpolation of a box field (cell centres (j - M/2 + 1/2) h) at points (x, y)."""
    m = field.shape[0]
    out = np.empty(len(pts))
    for q, (x, y) in enumerate(pts):
        gx, gy = x / h + m / 2 - 0.5, y / h + m / 2 - 0.5
        ix, iy = int(np.floor(gx)), int(np.floor(gy))
        wx, wy = keys_weights(gx - ix), keys_weights(gy - iy)
        block = field[iy - 1:iy + 3, ix - 1:ix + 3]   # rows y, columns x
        out[q] = wy @ block @ wx
    return out


def padded_source(geom, f) -> tuple[np.ndarray, int]:
    """The masked fine image in the centre of the box; returns (box field, M)."""
    ns = geom.n
    h = 2.0 / ns
    t_last = geom.n_t * geom.dt
    m = box_side(ns, geom.det_r, geom.support_r, geom.c, t_last)
    xc = -1.0 + (np.arange(ns) + 0.5) * h
    mask = (xc[None, :] ** 2 + xc[:, None] ** 2) < geom.support_r ** 2
    box = np.zeros((m, m))
    off = (m - ns) // 2
    box[off:off + ns, off:off + ns] = np.where(mask, np.asarray(f, dtype=np.float64), 0.0)
    return box, m


def wavenumbers(m: int, h: float) -> np.ndarray:
    """|k| of the box's FFT bins (rows y, columns x)."""
    k1 = 2.0 * np.pi * np.fft.fftfreq(m, d=h)
    return np.sqrt(k1[None, :] ** 2 + k1[:, None] ** 2)


def simulate(geom, f, times=None) -> np.ndarray:
    """Data [D][T] of the fine image f ([N_s][N_s], rows y) at times t_j = j dt
    (or the given times)."""
    box, m = padded_source(geom, f)
    h = 2.0 / geom.n
    th = np.asarray(geom.det_angles())
    pts = np.stack([geom.det_r * np.cos(th), geom.det_r * np.sin(th)], axis=1)
    ts = geom.times() if times is None else np.asarray(times, dtype=np.float64)
    spec = np.fft.fft2(box)
    kk = wavenumbers(m, h)
    out = np.empty((len(pts), len(ts)))
    for j, t in enumerate(ts):
        p = np.fft.ifft2(spec * np.cos(geom.c * kk * t)).real
        out[:, j] = sample(p, h, pts)
    return out
