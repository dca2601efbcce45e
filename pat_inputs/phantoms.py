"""Seeded synthetic phantoms and measurement noise.

Recipe (all draws from numpy.random.Generator(PCG64(seed)), in this order):
  * blobs: for each blob, u1, u2 ~ U[0,1) give an area-uniform centre in r < 0.7
    (r = 0.7 sqrt(u1), phi = 2 pi u2); then sigma ~ U[0.03, 0.1], a ~ U[0.5, 1];
    value a * exp(-|x - c|^2 / (2 sigma^2));
  * discs: centre drawn the same way, radius 0.15, value 1 inside;
  * line segments (vessel-like edges): two endpoints drawn the same way, value 1
    on pixels whose centre lies within distance h of the segment (about 2 px wide);
  * components are summed at the pixel centres, then set to 0 where r >= 0.9.
Noise: delta = eta * max|g| * N(0,1) i.i.d., drawn from a separate generator
seeded with seed + 10**6 (additive Gaussian noise, eq. (3)).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass(frozen=True)
class Blob:
    cx: float
    cy: float
    sigma: float
    amp: float


@dataclass(frozen=True)
class Disc:
    cx: float
    cy: float
    radius: float = 0.15
    value: float = 1.0


@dataclass(frozen=True)
class Line:
    x0: float
    y0: float
    x1: float
    y1: float
    value: float = 1.0


@dataclass
class PhantomSpec:
    blobs: List[Blob] = field(default_factory=list)
    discs: List[Disc] = field(default_factory=list)
    lines: List[Line] = field(default_factory=list)
    cutoff_r: float = 0.9


def pixel_centres(n: int):
    """Cell-centred coordinates: x_j = -1 + (j + 1/2) h (column j),
    y_i = -1 + (i + 1/2) h (row i), h = 2/n.  Returns (X, Y) of shape (n, n)."""
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")  # X[i, j] = x_j, Y[i, j] = y_i
    return X, Y


def _centre(rng, rmax=0.7):
    u1, u2 = rng.random(2)
    r = rmax * np.sqrt(u1)
    phi = 2 * np.pi * u2
    return float(r * np.cos(phi)), float(r * np.sin(phi))


def draw_phantom(n_blobs: int, n_discs: int, n_lines: int, seed: int) -> PhantomSpec:
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = PhantomSpec()
    for _ in range(n_blobs):
        cx, cy = _centre(rng)
        sigma = float(rng.uniform(0.03, 0.1))
        amp = float(rng.uniform(0.5, 1.0))
        spec.blobs.append(Blob(cx, cy, sigma, amp))
    for _ in range(n_discs):
        cx, cy = _centre(rng)
        spec.discs.append(Disc(cx, cy))
    for _ in range(n_lines):
        x0, y0 = _centre(rng)
        x1, y1 = _centre(rng)
        spec.lines.append(Line(x0, y0, x1, y1))
    return spec


def render_phantom(spec: PhantomSpec, n: int) -> np.ndarray:
    """Point-sample the phantom at the pixel centres; float64 (n, n), row i = y_i."""
    X, Y = pixel_centres(n)
    h = 2.0 / n
    f = np.zeros((n, n))
    for b in spec.blobs:
        f += b.amp * np.exp(-((X - b.cx) ** 2 + (Y - b.cy) ** 2) / (2 * b.sigma ** 2))
    for d in spec.discs:
        f += np.where((X - d.cx) ** 2 + (Y - d.cy) ** 2 < d.radius ** 2, d.value, 0.0)
    for ln in spec.lines:
        vx, vy = ln.x1 - ln.x0, ln.y1 - ln.y0
        L2 = vx * vx + vy * vy
        t = np.clip(((X - ln.x0) * vx + (Y - ln.y0) * vy) / max(L2, 1e-300), 0.0, 1.0)
        dist2 = (X - ln.x0 - t * vx) ** 2 + (Y - ln.y0 - t * vy) ** 2
        f += np.where(dist2 <= h * h, ln.value, 0.0)
    f[X * X + Y * Y >= spec.cutoff_r ** 2] = 0.0
    return f


def make_phantom(n: int, n_blobs: int, n_discs: int, n_lines: int, seed: int) -> np.ndarray:
    return render_phantom(draw_phantom(n_blobs, n_discs, n_lines, seed), n)


def add_noise(g: np.ndarray, eta: float, seed: int) -> np.ndarray:
    """g + eta * max|g| * N(0, 1), noise stream seeded with seed + 10**6."""
    if eta == 0.0:
        return np.array(g, copy=True)
    rng = np.random.Generator(np.random.PCG64(seed + 10 ** 6))
    return g + eta * float(np.max(np.abs(g))) * rng.standard_normal(g.shape)
