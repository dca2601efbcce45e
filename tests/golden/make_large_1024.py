"""Stored FP64 oracle values for the 1024^2 workload, and oracle timings.

Writes, from the oracle alone (the FP64 direct sums of oracle/) and the seeded
generators of pat_inputs:

* large_1024.npz -- the 1024^2 workload (1024 detectors on a 270 degree arc,
  2048 samples on (0, 2]):
    g_rows  A f at every 16th detector (64 full traces), f the seed-5000
            phantom (20 blobs, 3 discs, 4 lines: the workload's broadband
            instance 0);
    det     the detector indices of g_rows;
    pix     4000 flat pixel indices inside the support (seed 5002);
    a_pix   A* d at those pixels, d = standard normal (D, T) from seed 5100;
  with the wall time and thread count of each sum in large_1024.json.
* oracle_timings.json -- wall time of one A and one A* at the gradient-check
  shape, the 64^2 and both 256^2 workloads, and of one A at the 760^2 shape of
  the paper's timed run (Sec. 4.3), with the thread count.

Usage:  python tests/golden/make_large_1024.py [--golden] [--timings] [--threads T]
(no flag: both).  The 1024^2 forward takes minutes on a few cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from pat_inputs import config_geometry, make_phantom  # noqa: E402
from pat_inputs.geometry import paper_shape_geometry  # noqa: E402

DET_STRIDE = 16
N_PIX = 4000
SEED_F, SEED_D, SEED_PIX = 5000, 5100, 5002


def large_inputs(geom):
    """The phantom, datum and pixel sample the stored values are computed on."""
    f = make_phantom(geom.n, 20, 3, 4, SEED_F)
    d = np.random.default_rng(SEED_D).standard_normal((geom.n_det, geom.n_t))
    X = -1 + (np.arange(geom.n) + 0.5) * geom.h
    inside = ((X[None, :] ** 2 + X[:, None] ** 2) < geom.support_r ** 2).ravel()
    pix = np.sort(np.random.default_rng(SEED_PIX).choice(np.flatnonzero(inside), N_PIX, replace=False))
    return f, d, pix.astype(np.int64)


def cpu_name():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make_golden():
    geom = config_geometry(5)
    f, d, pix = large_inputs(geom)
    t0 = time.time()
    g = oracle.forward(geom, f)
    t_fwd = time.time() - t0
    det = np.arange(0, geom.n_det, DET_STRIDE)
    t0 = time.time()
    a_pix = oracle.adjoint_pixels(geom, d, pix)
    t_adj = time.time() - t0
    np.savez_compressed(os.path.join(HERE, "large_1024.npz"), g_rows=g[det], det=det, pix=pix, a_pix=a_pix)
    meta = dict(workload="1024x1024, 1024 detectors on a 270 deg arc, 2048 samples on (0,2]",
                phantom_seed=SEED_F, datum_seed=SEED_D, pixel_seed=SEED_PIX, det_stride=DET_STRIDE,
                n_pix=N_PIX, threads=oracle.get_threads(), cpu=cpu_name(),
                forward_s=round(t_fwd, 2), adjoint_pixels_s=round(t_adj, 2),
                g_norm=float(np.linalg.norm(g)), g_max=float(np.abs(g).max()))
    with open(os.path.join(HERE, "large_1024.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
        fh.write("\n")
    print(json.dumps(meta), flush=True)


def make_timings():
    shapes = [("gradcheck 32^2, 32 det on 120 deg, 64 samples", config_geometry("gradcheck"), True),
              ("64^2, 64 det on 360 deg, 128 samples", config_geometry(1), True),
              ("limited view 256^2, 256 det on 180 deg, 512 samples", config_geometry(2), True),
              ("256^2, 128 det on 120 deg, 512 samples", config_geometry(3), True),
              ("paper shape 760^2, 256 det on 270 deg, 2030 samples", paper_shape_geometry(), False)]
    rows = []
    for name, geom, both in shapes:
        f = make_phantom(geom.n, 5, 1, 0, 7)
        d = np.random.default_rng(7).standard_normal((geom.n_det, geom.n_t))
        t0 = time.time()
        oracle.forward(geom, f)
        tf = time.time() - t0
        ta = None
        if both:
            t0 = time.time()
            oracle.adjoint(geom, d)
            ta = time.time() - t0
        row = dict(workload=name, forward_s=round(tf, 3), adjoint_s=None if ta is None else round(ta, 3))
        print(json.dumps(row), flush=True)
        rows.append(row)
    out = dict(threads=oracle.get_threads(), cpu=cpu_name(), rows=rows)
    with open(os.path.join(HERE, "oracle_timings.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--golden", action="store_true")
    ap.add_argument("--timings", action="store_true")
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads > 0:
        oracle.set_threads(a.threads)
    both = not (a.golden or a.timings)
    if a.timings or both:
        make_timings()
    if a.golden or both:
        make_golden()


if __name__ == "__main__":
    main()
