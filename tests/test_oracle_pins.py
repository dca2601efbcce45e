"""Pins of the FP64 oracle against facts it does not compute itself.

Each test checks the oracle's direct sums against something independent:
closed forms (Gaussian Fourier transform and J_0 averages), numpy's FFT,
scipy's Bessel functions (mode form), continuum solutions of eq. (1)
(Hankel integral and 2D Poisson formula), symmetries of the geometry, the
detector coverages printed in Sec. 2.1 / 2.4.2, and sizes derived by hand.
A plausible slip (dropped W_n, wrong Fourier sign, swapped x/y, wrong time or
detector grid, wrong sign of the kappa term) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special

from pat_inputs import Blob, Geometry, PhantomSpec, config_geometry, render_phantom, pixel_centres

HERE = os.path.dirname(os.path.abspath(__file__))


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _small_geom(**kw):
    base = dict(n=24, n_det=20, n_t=40, dt=2.0 / 40, arc_span=200 * math.pi / 180)
    base.update(kw)
    return Geometry(**base)


# --- sizes ------------------------------------------------------------------

@pytest.mark.parametrize("cfg,expect", [
    # config 1: T=128 -> M = 2T = 256 = 2^8; dlam = pi/(256*1*(2/128)) = pi/4;
    # n_lam = floor(M c dt / h) = 256*(1/64)/(1/32) = 128; z = 128*pi/4 = 100.53,
    # z + 10 z^(1/3) = 147.03 -> K = 148; 2K+2 = 298 -> 324 = 4*81.
    (1, dict(M=256, n_lam=128, K=148, n_psi=324)),
    # config 2: M = 1024 = 2^10; n_lam = 1024*(2/512)/(2/256) = 512; z = 402.12,
    # z + 10 z^(1/3) = 475.93 -> K = 476; 2K+2 = 954 -> 972 = 4*243.
    (2, dict(M=1024, n_lam=512, K=476, n_psi=972)),
    # gradcheck: M = 128; n_lam = 64; z = 16 pi = 50.27 -> 87.17 -> K = 88; 178 -> 192.
    ("gradcheck", dict(M=128, n_lam=64, K=88, n_psi=192)),
    # config 5: M = 4096; n_lam = 2048; z = 512 pi = 1608.5 -> 1725.7 -> K = 1726; 3454 -> 3456.
    (5, dict(M=4096, n_lam=2048, K=1726, n_psi=3456)),
])
def test_sizes_by_hand(oracle_mod, cfg, expect):
    s = oracle_mod.sizes(config_geometry(cfg))
    for k, v in expect.items():
        assert s[k] == v, (k, s[k], v)
    assert abs(s["dlam"] - math.pi / 4) < 1e-15
    assert abs(s["kappa"] - (math.pi / 4) ** 2 / (24 * math.pi)) < 1e-15


def test_invalid_geometry_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.sizes(_small_geom(arc_span=7.0))
    with pytest.raises(ValueError):
        oracle_mod.sizes(_small_geom(support_r=1.5))
    with pytest.raises(ValueError):
        oracle_mod.sizes(_small_geom(dt=-1.0))


def test_detector_coverage_matches_paper():
    """Detector pitch alpha/D with coverage D * alpha/D reproduces the printed
    sub-array coverages (170 -> 179.30 deg, 112 -> 118.125 deg)."""
    gold = json.load(open(os.path.join(HERE, "golden", "detector_coverage.json")))
    pitch = gold["full_array"]["coverage_deg"] / gold["full_array"]["elements"]
    for sub in gold["subsets"]:
        D = sub["detectors"]
        geom = Geometry(n=8, n_det=D, n_t=4, dt=0.5, arc_span=math.radians(D * pitch))
        th = np.degrees(geom.det_angles())
        coverage = (th[-1] - th[0]) + (th[1] - th[0])  # D spacings of alpha/D
        assert round(coverage, sub["printed_digits"]) == pytest.approx(sub["coverage_deg"], abs=1e-9)
        assert np.allclose(np.diff(th), pitch)


# --- adjointness and linearity ----------------------------------------------

def test_dot_product_adjoint(oracle_mod):
    rng = np.random.default_rng(11)
    g = _small_geom()
    f = rng.standard_normal((g.n, g.n))
    d = rng.standard_normal((g.n_det, g.n_t))
    Af = oracle_mod.forward(g, f)
    Ad = oracle_mod.adjoint(g, d)
    err = abs(np.sum(Af * d) - np.sum(f * Ad)) / (np.linalg.norm(Af) * np.linalg.norm(d))
    assert err < 1e-12


def test_linearity(oracle_mod):
    rng = np.random.default_rng(12)
    g = _small_geom(em_correction=1)
    f1, f2 = rng.standard_normal((2, g.n, g.n))
    lhs = oracle_mod.forward(g, 2.0 * f1 - 3.0 * f2)
    rhs = 2.0 * oracle_mod.forward(g, f1) - 3.0 * oracle_mod.forward(g, f2)
    assert _rel(lhs, rhs) < 1e-13


def test_adjoint_pixels_agrees_with_full(oracle_mod):
    rng = np.random.default_rng(13)
    g = _small_geom()
    d = rng.standard_normal((g.n_det, g.n_t))
    full = oracle_mod.adjoint(g, d).ravel()
    idx = np.array([0, 5, 100, 287, 300, 575])
    assert np.allclose(oracle_mod.adjoint_pixels(g, d, idx), full[idx], rtol=1e-12, atol=1e-14)


# --- step 1: Fourier sign, pixel grid, mask ---------------------------------

def test_polar_rays_equal_numpy_fft(oracle_mod):
    """psi = 0 and psi = pi/2 rays of step 1 equal numpy's FFT of the column /
    row sums zero-padded to P = 2 pi/(dlam h) = 4N points, times the phase of
    the half-pixel offset: F(n,0) = h^2 e^{i n dlam (1 - h/2)} FFT_P(s)[n]."""
    g = config_geometry(1)  # dlam h = pi/128 -> P = 256 = 4N
    s = oracle_mod.sizes(g)
    rng = np.random.default_rng(14)
    X, Y = pixel_centres(g.n)
    f = rng.standard_normal((g.n, g.n))
    mf = np.where(X * X + Y * Y < g.support_r ** 2, f, 0.0)
    F = oracle_mod.polar_spectrum(g, f)
    h, P = g.h, 4 * g.n
    n = np.arange(1, s["n_lam"] + 1)
    phase = np.exp(1j * n * s["dlam"] * (1 - h / 2))
    ray0 = h * h * phase * np.fft.fft(mf.sum(axis=0), P)[n]        # sum over rows -> function of x_j
    ray90 = h * h * phase * np.fft.fft(mf.sum(axis=1), P)[n]       # sum over columns -> function of y_i
    assert _rel(F[:, 0], ray0) < 1e-12
    assert _rel(F[:, s["n_psi"] // 4], ray90) < 1e-12
    # real image: antipodal points are complex conjugates
    assert _rel(F[:, s["n_psi"] // 2], np.conj(ray0)) < 1e-12


def _gauss_blobs(h):
    return [Blob(0.1, -0.05, 3 * h, 1.0), Blob(-0.2, 0.15, 3 * h, 0.7)]


def test_gaussian_closed_form_forward(oracle_mod):
    from oracle import reference as ref
    g = Geometry(n=64, n_det=16, n_t=128, dt=2 / 128, arc_span=math.radians(270))
    blobs = _gauss_blobs(g.h)
    f = render_phantom(PhantomSpec(blobs=blobs, cutoff_r=10.0), g.n)
    s = oracle_mod.sizes(g)
    A = oracle_mod.forward(g, f)
    C = ref.discrete_gaussian_data(g, s, blobs)
    assert _rel(A, C) < 1e-12
    # without the endpoint term as well
    g0 = g.with_(em_correction=0)
    s0 = oracle_mod.sizes(g0)
    assert _rel(oracle_mod.forward(g0, f), ref.discrete_gaussian_data(g0, s0, blobs)) < 1e-12


def test_impulse_closed_form_adjoint(oracle_mod):
    from oracle import reference as ref
    g = Geometry(n=48, n_det=12, n_t=96, dt=2 / 96, arc_span=math.radians(180))
    s = oracle_mod.sizes(g)
    for (d, j) in [(0, 10), (7, 60), (11, 95)]:
        data = np.zeros((g.n_det, g.n_t))
        data[d, j] = 1.0
        A = oracle_mod.adjoint(g, data)
        C = ref.discrete_impulse_adjoint(g, s, d, j)
        assert np.abs(A - C).max() < 1e-12 * np.abs(C).max()


# --- steps 2-5: mode form (Bessel functions, FFT) = plane-wave form ----------

def test_mode_form_equals_plane_wave_form(oracle_mod):
    """Steps 2-5 through angular Fourier modes, i^k J_k(lam R) weights (scipy)
    and numpy's FFT equal the oracle's plane-wave sums (Jacobi-Anger)."""
    g = Geometry(n=32, n_det=24, n_t=64, dt=2 / 64, arc_span=math.radians(150), arc_center=0.3)
    s = oracle_mod.sizes(g)
    rng = np.random.default_rng(15)
    F = rng.standard_normal((s["n_lam"], s["n_psi"])) + 1j * rng.standard_normal((s["n_lam"], s["n_psi"]))
    mass = 0.37
    K, NP = s["K"], s["n_psi"]
    lam = np.arange(1, s["n_lam"] + 1) * s["dlam"]
    W = lam * s["dlam"] / (2 * math.pi)
    Fk = np.fft.fft(F, axis=1) / NP                      # F_k for k = 0..NP-1 (negative k wrap)
    ks = np.arange(-K, K + 1)
    b = (1j ** ks)[None, :] * special.jv(ks[None, :], lam[:, None] * g.det_r) * W[:, None] * Fk[:, ks % NP]
    t = np.asarray(g.times())
    Bk = np.cos(g.c * np.outer(t, lam)) @ b                # (T, 2K+1)
    th = np.asarray(g.det_angles())
    E = np.exp(1j * np.outer(th, ks))                     # (D, 2K+1)
    mode = np.real(E @ Bk.T) + s["kappa"] * mass
    plane = oracle_mod.polar_to_data(g, F, mass)
    assert _rel(plane, mode) < 1e-12


# --- symmetries ---------------------------------------------------------------

def test_rotation_by_90_degrees(oracle_mod):
    """Rotating the image by +90 deg (f'(x,y) = f(y,-x), i.e. np.rot90(f, -1)) and
    the detector arc by +pi/2 leaves the data unchanged (Npsi % 4 == 0)."""
    rng = np.random.default_rng(16)
    g = _small_geom(arc_center=0.4)
    f = rng.standard_normal((g.n, g.n))
    a = oracle_mod.forward(g, f)
    b = oracle_mod.forward(g.with_(arc_center=0.4 + math.pi / 2), np.rot90(f, -1))
    assert _rel(b, a) < 1e-12
    # adjoint commutes the same way
    d = rng.standard_normal((g.n_det, g.n_t))
    fa = oracle_mod.adjoint(g, d)
    fb = oracle_mod.adjoint(g.with_(arc_center=0.4 + math.pi / 2), d)
    assert _rel(fb, np.rot90(fa, -1)) < 1e-12


def test_mirror_y(oracle_mod):
    """f'(x,y) = f(x,-y) with the arc mirrored (theta -> -theta) gives the data
    with detectors in reverse order."""
    rng = np.random.default_rng(17)
    g = _small_geom(arc_center=0.4)
    f = rng.standard_normal((g.n, g.n))
    a = oracle_mod.forward(g, f)
    b = oracle_mod.forward(g.with_(arc_center=-0.4), np.flipud(f))
    assert _rel(b, a[::-1]) < 1e-12


# --- physics: continuum solution of eq. (1)-(2) --------------------------------

def test_continuum_references_agree():
    from oracle import reference as ref
    b = Blob(0.1, -0.05, 0.05, 0.8)
    for (x, y) in [(1.0, 0.0), (0.0, -1.0), (-0.6, 0.8)]:
        for t in [0.2, 0.7, 1.05, 1.6]:
            a1 = ref.hankel_gaussian(b, x, y, t)
            a2 = ref.poisson_gaussian(b, x, y, t)
            assert abs(a1 - a2) < 1e-9 * max(1.0, abs(a1))


def test_operator_converges_to_continuum(oracle_mod):
    """The discrete operator approaches the continuum pressure of eq. (1)-(2);
    the kappa term lowers the error, and raising the lambda oversampling
    sigma_t lowers it further (about 16x per doubling with kappa, 4x without)."""
    from oracle import reference as ref
    g = Geometry(n=64, n_det=8, n_t=128, dt=2 / 128, arc_span=math.radians(270))
    blobs = _gauss_blobs(g.h)
    f = render_phantom(PhantomSpec(blobs=blobs, cutoff_r=10.0), g.n)
    th = np.asarray(g.det_angles())
    cont = np.array([[sum(ref.hankel_gaussian(b, math.cos(a), math.sin(a), t) for b in blobs)
                      for t in g.times()] for a in th])
    errs = {}
    for st in (2.0, 4.0, 8.0):
        for em in (0, 1):
            A = oracle_mod.forward(g.with_(lambda_oversample=st, em_correction=em), f)
            errs[(st, em)] = _rel(A, cont)
    assert errs[(2.0, 1)] < 2.5e-3
    for st in (2.0, 4.0, 8.0):
        assert errs[(st, 1)] < errs[(st, 0)]
    assert errs[(4.0, 0)] < errs[(2.0, 0)] / 3 and errs[(8.0, 0)] < errs[(4.0, 0)] / 3
    assert errs[(4.0, 1)] < errs[(2.0, 1)] / 8 and errs[(8.0, 1)] < errs[(4.0, 1)] / 8
