"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every function include/pat.h declares; the
host-only routines (size derivation, Bessel table, status strings) and the
argument checks that run before any launch are exercised here.
"""
import ctypes
import math

import numpy as np
import pytest
from scipy import special

from pat_inputs import Geometry, config_geometry
from pat_inputs.geometry import paper_shape_geometry


@pytest.fixture(scope="module")
def patlib():
    from paper_2604_19176_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(patlib):
    lib = patlib.load()
    names = patlib.declared_functions()
    assert "pat_forward" in names and "pat_adjoint" in names and "pat_plan_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("cfg", [1, 2, 3, "gradcheck", 5])
def test_derived_sizes_match_oracle(patlib, oracle_mod, cfg):
    """The plan's size rules (implemented separately from the oracle's) agree."""
    import paper_2604_19176_amd as pat
    geom = config_geometry(cfg)
    info = pat.pat_plan_derive(pat.desc_from_geometry(geom))
    ref = oracle_mod.sizes(geom)
    assert (info.M, info.n_lam, info.K, info.n_psi) == (ref["M"], ref["n_lam"], ref["K"], ref["n_psi"])
    assert info.dlam == pytest.approx(ref["dlam"], rel=1e-15)
    assert info.kappa == pytest.approx(ref["kappa"], rel=1e-15)
    assert info.n_grid >= 2 * geom.n and info.n_grid % 2 == 0
    _check_synthesis(info, geom)


def _is_smooth23(p):
    while p % 2 == 0:
        p //= 2
    while p % 3 == 0:
        p //= 3
    return p == 1


def _check_synthesis(info, geom):
    """Synthesis over detector angles: one FFT of length P when dtheta = 2 pi s / P
    with P = 2^a 3^b (detectors at every s-th grid point), else the chirp-z."""
    turns = geom.arc_span / (2 * math.pi * geom.n_det)       # dtheta / (2 pi)
    D = geom.n_det
    if info.syn_stride:
        P, s = info.len_czt, info.syn_stride
        assert _is_smooth23(P) and P <= 8192 and math.gcd(s, P) == 1
        assert abs(P * turns - s) <= 1e-9 * s
        assert s * (D - 1) < P                       # detectors are distinct grid points
    else:
        assert info.syn_stride == 0
        assert info.len_czt >= info.K + D            # Bluestein chirp-z
        # no 2^a 3^b grid within the size limits carries the detectors
        for P in range(D, min(8192, 3 * info.len_czt) + 1):
            if _is_smooth23(P):
                assert abs(P * turns - round(P * turns)) > 1e-9 * P * turns or round(P * turns) == 0


@pytest.mark.parametrize("geom,P,s", [
    (config_geometry(1), 64, 1), (config_geometry(2), 512, 1), (config_geometry(3), 384, 1),
    (config_geometry(5), 4096, 3), (paper_shape_geometry(), 1024, 3),
    (Geometry(n=32, n_det=12, n_t=64, dt=2 / 64, arc_span=2 * math.pi * 24 / 27), 27, 2),
    (Geometry(n=40, n_det=37, n_t=75, dt=2.2 / 75, arc_span=math.radians(250)), 0, 0)])
def test_synthesis_grid(patlib, geom, P, s):
    """Known detector layouts: 270 degrees with D detectors is every third point of
    a 4D grid; 250 degrees over 37 detectors lies on no 2^a 3^b grid."""
    import paper_2604_19176_amd as pat
    info = pat.pat_plan_derive(pat.desc_from_geometry(geom))
    _check_synthesis(info, geom)
    if P:
        assert (info.len_czt, info.syn_stride) == (P, s)
    else:
        assert info.syn_stride == 0


def test_derived_sizes_random_geometries(patlib, oracle_mod):
    import paper_2604_19176_amd as pat
    rng = np.random.default_rng(3)
    for _ in range(40):
        n = int(rng.integers(16, 300))
        t = int(rng.integers(8, 900))
        geom = Geometry(n=n, n_det=int(rng.integers(1, 400)), n_t=t, dt=float(rng.uniform(0.5, 3.0)) / t,
                        arc_span=float(rng.uniform(0.1, 2 * math.pi)), c=float(rng.uniform(0.5, 2.0)),
                        lambda_oversample=float(rng.choice([1.0, 1.5, 2.0, 3.0])))
        try:
            ref = oracle_mod.sizes(geom)
        except ValueError:
            continue
        try:
            info = pat.pat_plan_derive(pat.desc_from_geometry(geom))
        except pat.PatError as e:
            assert e.status == pat._lib.PAT_ERR_UNSUPPORTED  # valid but beyond the kernels' limits
            continue
        assert (info.M, info.n_lam, info.K, info.n_psi) == (ref["M"], ref["n_lam"], ref["K"], ref["n_psi"])
        _check_synthesis(info, geom)


def _smooth23_at_least(x):
    return min(p for p in (2 ** a * 3 ** b for a in range(16) for b in range(10)) if p >= x)


def test_synthesis_grid_random_rational_arcs(patlib):
    """Arcs of D detectors with pitch 2 pi s / P (P = 2^a 3^b, gcd(s, P) = 1) use
    the P-point grid with stride s whenever P is within the size limits."""
    import paper_2604_19176_amd as pat
    rng = np.random.default_rng(12)
    smooth = [p for p in (2 ** a * 3 ** b for a in range(14) for b in range(9)) if 8 <= p <= 8192]
    seen = 0
    for _ in range(120):
        P = int(rng.choice(smooth))
        s = int(rng.integers(1, 8))
        if math.gcd(s, P) != 1 or P // s < 2:
            continue
        D = int(rng.integers(1, min(P // s, 600) + 1))
        geom = Geometry(n=32, n_det=D, n_t=64, dt=2 / 64, arc_span=2 * math.pi * s * D / P)
        info = pat.pat_plan_derive(pat.desc_from_geometry(geom))
        _check_synthesis(info, geom)
        L = _smooth23_at_least(info.K + D)
        if P <= min(8192, 3 * L):
            assert (info.len_czt, info.syn_stride) == (P, s), (P, s, D)
            seen += 1
    assert seen >= 20


@pytest.mark.parametrize("kw,status", [
    (dict(n=8), -2),                  # below the smallest supported grid
    (dict(arc_span=7.0), -1),
    (dict(arc_span=0.0), -1),
    (dict(dt=-1.0), -1),
    (dict(c=0.0), -1),
    (dict(support_r=1.2), -1),        # support outside the detector circle
    (dict(n_det=0), -1),
    (dict(lambda_oversample=0.5), -1),
    (dict(n_t=1, dt=1e-4), -1),       # no radial frequency below pi/h
    (dict(n_t=4096, dt=2 / 4096), -2),  # cosine FFT longer than the LDS plans
])
def test_plan_argument_errors(patlib, kw, status):
    import paper_2604_19176_amd as pat
    base = dict(n=32, n_det=16, n_t=64, dt=2 / 64)
    base.update(kw)
    geom = Geometry(**base)
    with pytest.raises(pat.PatError) as ei:
        pat.pat_plan_derive(pat.desc_from_geometry(geom))
    assert ei.value.status == status


def test_bessel_table_matches_scipy(patlib):
    import paper_2604_19176_amd as pat
    for x in [1e-3, 0.785, 7.0, 99.5, 402.12, 1608.5]:
        kmax = int(math.ceil(x + 10 * x ** (1 / 3))) + 3
        got = np.array(pat.pat_bessel_jn_table(kmax, x))
        ref = special.jv(np.arange(kmax + 1), x)
        assert np.abs(got - ref).max() < 1e-13, x


def test_status_strings(patlib):
    import paper_2604_19176_amd as pat
    assert pat.pat_status_string(0) == "ok"
    for s in (-1, -2, -3, -4, -5):
        assert pat.pat_status_string(s) not in ("ok", "unknown status")
    assert pat.pat_status_string(7) == "unknown status"


def test_calls_reject_null_arguments_before_launch(patlib):
    """Host checks return PAT_ERR_ARG without touching a GPU."""
    lib = patlib.load()
    one = ctypes.c_void_p(1)
    assert lib.pat_forward(None, one, one, 1, one, 0, None) == -1
    assert lib.pat_adjoint(None, one, one, 1, one, 0, None) == -1
    assert lib.pat_tv_grad(None, one, None, 16, 1, 1e-3, None) == -1
    assert lib.pat_tv_grad(one, one, None, 1, 1, 1e-3, None) == -1
    assert lib.pat_tv_grad(one, one, None, 16, 1, 0.0, None) == -1
    assert lib.pat_pgd_update(None, one, None, 10, 0.1, 0.1, None) == -1
    assert lib.pat_residual(one, None, None, 10, 1, None) == -1
    assert lib.pat_workspace_size(None, 1) == 0
    assert lib.pat_plan_query(None, None) == -1
    lib.pat_plan_destroy(None)  # no-op


def test_batch_and_tuner_entry_points_reject_null_arguments(patlib):
    """The launch-shape, batch and autotuner entry points check their
    arguments on the host before any HIP call."""
    lib = patlib.load()
    one = ctypes.c_void_p(1)
    cfg = patlib.pat_launch()
    assert lib.pat_plan_get_launch(None, ctypes.byref(cfg)) == -1
    assert lib.pat_plan_set_launch(None, ctypes.byref(cfg)) == -1
    split = ctypes.c_int(-7)
    assert lib.pat_plan_set_split(None, 2) == -1
    assert lib.pat_plan_get_split(None, ctypes.byref(split)) == -1
    assert split.value == -7
    out = ctypes.c_void_p()
    assert lib.pat_batch_create(None, 1, ctypes.byref(out)) == -1
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.pat_batch_create(arr, 2, ctypes.byref(out)) == -1     # NULL plans
    assert lib.pat_batch_create(arr, 0, ctypes.byref(out)) == -1     # empty batch
    assert out.value is None
    assert lib.pat_batch_workspace_size(None) == 0
    assert lib.pat_batch_forward(None, one, one, one, 1 << 20, None) == -1
    assert lib.pat_batch_adjoint(None, one, one, one, 1 << 20, None) == -1
    assert lib.pat_batch_get_launch(None, ctypes.byref(cfg)) == -1
    assert lib.pat_batch_set_launch(None, ctypes.byref(cfg)) == -1
    assert lib.pat_autotune_plan(None, 1, None) == -1
    assert lib.pat_autotune_batch(None, None) == -1
    lib.pat_batch_destroy(None)  # no-op


def test_explicit_angles_select_the_dense_synthesis(patlib):
    """Explicit detector angles (host array in the descriptor) give syn_dense = 1
    with the same radial/angular sizes as the uniform arc; a non-finite angle is
    rejected before any allocation."""
    import paper_2604_19176_amd as pat
    g = Geometry(n=48, n_det=20, n_t=96, dt=2 / 96, arc_span=math.radians(90))
    ge = g.with_(det_theta=tuple(np.random.default_rng(1).uniform(-3, 3, 20)))
    iu = pat.pat_plan_derive(pat.desc_from_geometry(g))
    ie = pat.pat_plan_derive(pat.desc_from_geometry(ge))
    assert (iu.syn_dense, ie.syn_dense) == (0, 1)
    assert (ie.len_czt, ie.syn_stride) == (0, 0)
    assert (ie.M, ie.n_lam, ie.K, ie.n_psi) == (iu.M, iu.n_lam, iu.K, iu.n_psi)
    bad = g.with_(det_theta=tuple([0.0] * 19 + [float("nan")]))
    with pytest.raises(pat.PatError) as e:
        pat.pat_plan_derive(pat.desc_from_geometry(bad))
    assert e.value.status == patlib.PAT_ERR_ARG


def test_python_layer_rejects_mismatched_tensors():
    """The binding checks shapes before it hands raw pointers to the library:
    an output of the wrong batch, or elementwise operands of different shapes,
    raise ValueError on the host (the C-ABI cannot see buffer sizes)."""
    import torch
    import paper_2604_19176_amd as pat
    with pytest.raises(ValueError):
        pat._check_out(torch.zeros(3, 32, 64), "out", (2, 32, 64), None)   # batch 3 for a batch-2 call
    with pytest.raises(ValueError):
        pat._check_out(torch.zeros(32, 64), "out", (2, 32, 64), None)      # unbatched out, batched call
    f = torch.zeros(2, 16, 16)
    with pytest.raises(ValueError):
        pat.pgd_update(f, torch.zeros(16, 16), None, 0.1, 0.0)
    with pytest.raises(ValueError):
        pat.pgd_update(f, torch.zeros(2, 16, 16), torch.zeros(1, 16, 16), 0.1, 0.0)
    with pytest.raises(ValueError):
        pat.residual(torch.zeros(2, 8, 10), torch.zeros(2, 8, 11))
    with pytest.raises(ValueError):
        pat.residual(torch.zeros(8, 10), torch.zeros(1, 8, 10))
    # matching shapes still need GPU tensors
    with pytest.raises(ValueError):
        pat.pgd_update(f, torch.zeros(2, 16, 16), None, 0.1, 0.0)
    with pytest.raises((TypeError, ValueError)):
        pat.pgd_update(f, torch.zeros(2, 16, 16, dtype=torch.float64), None, 0.1, 0.0)
