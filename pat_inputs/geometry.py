"""Geometry descriptors of the measured workloads.

A `Geometry` names the physical set-up of eq. (1)-(2) (Sec. 2.1): an N x N
image grid of cell-centred pixels on [-1, 1]^2, D detectors spread uniformly
over an arc of a circle of radius R (theta_d = theta_c - alpha/2 +
(d + 1/2) alpha / D, so D detectors cover D * alpha/D; with 270/256 degrees per
element this reproduces the 170 -> 179.3 deg and 112 -> 118.125 deg sub-arrays
of Sec. 2.1 / 2.4.2), T time samples t_j = j * dt (j = 1..T) and a constant
speed of sound c.  Both the GPU library and the oracle take these fields.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace
from typing import Optional, Tuple


@dataclass(frozen=True)
class Geometry:
    n: int                      # grid side N
    n_det: int                  # D
    n_t: int                    # T
    dt: float                   # time step; t_j = j * dt, j = 1..T
    arc_span: float = 2 * math.pi   # alpha in (0, 2 pi]
    arc_center: float = -math.pi / 2  # theta_c (array at the bottom)
    c: float = 1.0
    support_r: float = 1.0      # rho_s: pixels with x^2 + y^2 >= rho_s^2 are dropped
    det_r: float = 1.0          # R
    lambda_oversample: float = 2.0
    em_correction: int = 1
    # explicit detector angles theta_d [rad] (D values, any order and spacing);
    # None: the uniform arc above
    det_theta: Optional[Tuple[float, ...]] = None

    def __post_init__(self):
        if self.det_theta is not None:
            object.__setattr__(self, "det_theta", tuple(float(t) for t in self.det_theta))
            if len(self.det_theta) != self.n_det:
                raise ValueError("det_theta needs n_det = %d angles" % self.n_det)

    def asdict(self):
        return asdict(self)

    def with_(self, **kw) -> "Geometry":
        return replace(self, **kw)

    @property
    def h(self) -> float:
        return 2.0 / self.n

    def det_angles(self):
        if self.det_theta is not None:
            return list(self.det_theta)
        a, D = self.arc_span, self.n_det
        return [self.arc_center - a / 2 + (d + 0.5) * a / D for d in range(D)]

    def times(self):
        return [(j + 1) * self.dt for j in range(self.n_t)]


def _deg(x):
    return x * math.pi / 180.0


def _geom(n, d, t, arc_deg, tmax=2.0, **kw):
    return Geometry(n=n, n_det=d, n_t=t, dt=tmax / t, arc_span=_deg(arc_deg), **kw)


# Workload table.  `phantom` gives (blobs, discs, lines); `noise` is eta, the
# noise standard deviation as a fraction of max|A f|.
CONFIGS = {
    # plain forward+adjoint: 64^2, 64 detectors on the full circle, 128 samples
    1: dict(geom=_geom(64, 64, 128, 360.0), phantom=(5, 1, 0), noise=0.0, seed=1, batch=1),
    # limited view: 256^2, 256 detectors on a 180 degree arc, 512 samples, 1 % noise
    2: dict(geom=_geom(256, 256, 512, 180.0), phantom=(20, 3, 4), noise=0.01, seed=2, batch=1),
    # differentiation: 256^2, 128 detectors on a 120 degree arc, 512 samples, 2 % noise
    3: dict(geom=_geom(256, 128, 512, 120.0), phantom=(20, 3, 4), noise=0.02, seed=3, batch=1,
            tv_lambda=1e-3, tv_steps=500),
    # gradient check shape: 32^2, 32 detectors on 120 degrees, 64 samples
    "gradcheck": dict(geom=_geom(32, 32, 64, 120.0), phantom=(5, 1, 0), noise=0.0, seed=33, batch=1),
    # large: 1024^2, 1024 detectors on 270 degrees, 2048 samples, batch 8, 1 % noise
    5: dict(geom=_geom(1024, 1024, 2048, 270.0), phantom=(20, 3, 4), noise=0.01, seed=5000, batch=8,
            tv_steps=2000),
}


def config_geometry(cfg) -> Geometry:
    return CONFIGS[cfg]["geom"]


def mixed_batch_geometries(count: int = 64):
    """The heterogeneous batch: instance b has N = (128, 256, 512)[b % 3],
    D = (64, 128, 256, 512)[(b // 3) % 4], arc = (90, 180, 360)[(b // 12) % 3]
    degrees and T = 2N; seeds 4000 + b."""
    out = []
    for b in range(count):
        n = (128, 256, 512)[b % 3]
        d = (64, 128, 256, 512)[(b // 3) % 4]
        arc = (90.0, 180.0, 360.0)[(b // 12) % 3]
        out.append((_geom(n, d, 2 * n, arc), 4000 + b))
    return out


def paper_shape_geometry() -> Geometry:
    """The shape of the paper's timed workload (Sec. 4.3 / 2.4.2): a 760^2
    grid, 256 detectors on 270 degrees, 2030 time samples."""
    return _geom(760, 256, 2030, 270.0)


def jittered_array_geometry(n: int = 256, n_det: int = 256, n_t: int = 512, arc_deg: float = 180.0,
                            jitter: float = 0.3, seed: int = 2) -> Geometry:
    """The limited-view workload's array with each element displaced along the
    circle by a uniform draw in [-jitter, jitter] element pitches (seeded):
    a non-uniform array whose angles only the dense synthesis handles."""
    import numpy as np
    g = _geom(n, n_det, n_t, arc_deg)
    pitch = g.arc_span / n_det
    th = np.asarray(g.det_angles()) + pitch * np.random.default_rng(seed).uniform(-jitter, jitter, n_det)
    return g.with_(det_theta=tuple(th))
