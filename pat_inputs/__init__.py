"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module holds the geometry descriptors of the benchmark workloads and the
seeded phantom / noise generators.  It contains none of the operator's
arithmetic: it only describes *what* is measured (grid, detectors, time
samples, speed of sound) and draws images and noise.

Workloads stand in for the paper's data sets (the simulated phantoms of
Sec. 2.4.1, the digital-twin phantoms of Sec. 2.4.2 and the mouse data of
Sec. 2.4.3 are not available): images of Gaussian blobs, uniform discs and thin
vessel-like line segments inside the disc r < 0.9, detectors on a circle of
radius 1 restricted to an arc (limited view, Sec. 2.1), time samples uniform
on (0, 2].
"""
from .geometry import Geometry, CONFIGS, config_geometry, paper_shape_geometry  # noqa: F401
from .phantoms import (  # noqa: F401
    Blob, Disc, Line, PhantomSpec, draw_phantom, render_phantom, make_phantom,
    add_noise, pixel_centres,
)
