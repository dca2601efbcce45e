"""Pins of the FP64 wave-propagation simulator reference (oracle/simulate.py)
against facts fixed independently of it: Keys interpolation's reproduction of
quadratics, the identity at t = 0, the exact 2D solution for a Gaussian
initial pressure (a Hankel-transform integral by quadrature), the grid's 90
degree rotation symmetry and the box's wrap-free margin."""
import math

import numpy as np
import pytest

from oracle import simulate as sim
from pat_inputs import Geometry


def test_box_rule_and_smooth_lengths():
    assert [sim.smooth_2a3b(m) for m in (1, 5, 7, 17, 100, 1025)] == [1, 6, 8, 18, 108, 1152]
    for ns, r, t in [(32, 1.0, 2.0), (96, 1.0, 1.0), (512, 1.0, 2.0), (48, 0.5, 0.25)]:
        m = sim.box_side(ns, r, 1.0, 1.0, t)
        h = 2.0 / ns
        half = m * h / 2
        assert m % 2 == 0 and (m - ns) % 2 == 0 and m >= ns
        assert 2 * half - r - 1.0 > t and half > r + 3 * h
    assert sim.box_side(512, 1.0, 1.0, 1.0, 2.0) == 1152


@pytest.mark.parametrize("frac", [0.0, 0.13, 0.5, 0.77, 0.999])
def test_keys_weights_reproduce_quadratics(frac):
    w = sim.keys_weights(frac)
    off = np.array([-1.0, 0.0, 1.0, 2.0])
    assert abs(w.sum() - 1.0) < 1e-14
    assert abs(w @ off - frac) < 1e-14
    assert abs(w @ off ** 2 - frac ** 2) < 1e-14


def test_quadratic_image_at_time_zero():
    # detectors inside the support, where the image is the quadratic itself
    geom = Geometry(n=48, n_det=12, n_t=1, dt=0.1, det_r=0.5, arc_span=2 * math.pi)
    h = 2.0 / geom.n
    xc = -1.0 + (np.arange(geom.n) + 0.5) * h
    x, y = xc[None, :], xc[:, None]
    q = lambda x, y: 0.3 + 0.7 * x - 0.4 * y + 1.1 * x * x - 0.6 * x * y + 0.9 * y * y
    g = sim.simulate(geom, q(x, y), times=[0.0])
    th = np.asarray(geom.det_angles())
    ref = q(0.5 * np.cos(th), 0.5 * np.sin(th))
    assert np.max(np.abs(g[:, 0] - ref)) < 1e-12


def test_gaussian_against_the_exact_solution():
    from scipy.integrate import quad
    from scipy.special import j0
    sigma, c = 0.15, 1.3
    geom = Geometry(n=96, n_det=16, n_t=6, dt=0.3, arc_span=2 * math.pi, c=c)
    h = 2.0 / geom.n
    xc = -1.0 + (np.arange(geom.n) + 0.5) * h
    f = np.exp(-(xc[None, :] ** 2 + xc[:, None] ** 2) / sigma ** 2)
    g = sim.simulate(geom, f)
    # p(r, t) = (sigma^2 / 2) int_0^inf k exp(-sigma^2 k^2 / 4) cos(c k t) J0(k r) dk
    kmax = 12.0 / sigma
    ref = np.array([0.5 * sigma ** 2 * quad(lambda k: k * math.exp(-0.25 * sigma ** 2 * k * k) * math.cos(c * k * t)
                                              * j0(k * geom.det_r), 0.0, kmax, limit=400, epsabs=1e-13)[0]
                    for t in geom.times()])
    err = np.max(np.abs(g - ref[None, :])) / np.max(np.abs(ref))
    print("Gaussian: max error %.2e of max |p| %.3e" % (err, np.max(np.abs(ref))))
    assert err < 1e-3
    # radial symmetry: every detector on the circle sees the same trace
    assert np.max(np.abs(g - g[:1])) < 1e-3 * np.max(np.abs(ref))


def test_rotation_by_90_degrees():
    rng = np.random.default_rng(5)
    n = 40
    th = rng.uniform(0, 2 * math.pi, 9)
    f = rng.standard_normal((n, n))
    fr = np.empty_like(f)
    for i in range(n):
        for j in range(n):
            fr[i, j] = f[n - 1 - j, i]   # f'(x, y) = f(y, -x): the image turned by +90 degrees
    geom = Geometry(n=n, n_det=9, n_t=8, dt=0.2, det_theta=tuple(th))
    geom_r = geom.with_(det_theta=tuple(th + math.pi / 2))
    a, b = sim.simulate(geom, f), sim.simulate(geom_r, fr)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_larger_box_changes_nothing_but_the_discrete_tails():
    rng = np.random.default_rng(6)
    geom = Geometry(n=40, n_det=10, n_t=12, dt=2.0 / 12, arc_span=math.radians(270))
    h = 2.0 / geom.n
    xc = -1.0 + (np.arange(geom.n) + 0.5) * h
    # smooth blobs (well inside the band), so the discrete propagator's tails are small
    f = np.zeros((geom.n, geom.n))
    for _ in range(3):
        cx, cy = rng.uniform(-0.5, 0.5, 2)
        f += np.exp(-((xc[None, :] - cx) ** 2 + (xc[:, None] - cy) ** 2) / 0.2 ** 2)
    g = sim.simulate(geom, f)
    m = sim.box_side(geom.n, geom.det_r, geom.support_r, geom.c, geom.n_t * geom.dt)
    big = m + 48
    box = np.zeros((big, big))
    off = (big - geom.n) // 2
    mask = (xc[None, :] ** 2 + xc[:, None] ** 2) < 1.0
    box[off:off + geom.n, off:off + geom.n] = np.where(mask, f, 0.0)
    spec = np.fft.fft2(box)
    kk = sim.wavenumbers(big, h)
    th = np.asarray(geom.det_angles())
    pts = np.stack([np.cos(th), np.sin(th)], axis=1)
    g2 = np.stack([sim.sample(np.fft.ifft2(spec * np.cos(kk * t)).real, h, pts) for t in geom.times()], axis=1)
    err = np.max(np.abs(g - g2)) / np.max(np.abs(g2))
    print("box %d vs %d: max difference %.2e" % (m, big, err))
    assert err < 1e-3
