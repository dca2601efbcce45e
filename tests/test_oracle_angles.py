"""Pins of the FP64 oracle with explicit detector angles (CPU only).

The operator of eq. (1)-(3) does not depend on how the detector angles are
spaced; `Geometry.det_theta` replaces the uniform arc by D given angles.

* Gaussian blobs: the oracle's data at random, unsorted angles equal the
  closed form through J_0 (oracle.reference.discrete_gaussian_data), the same
  pin as for the uniform arc (1e-12).
* The uniform arc's own angles given explicitly reproduce the arc (1e-13).
* Permuting the angles permutes the rows of A f; the union of two arcs
  stacks the rows of the two arcs' operators.
* A* is the transpose (dot test, 1e-12) and the impulse closed form holds.
"""
import math

import numpy as np
import pytest

from pat_inputs import Blob, Geometry, PhantomSpec, render_phantom


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _random_angles(D, seed):
    return np.random.default_rng(seed).uniform(-math.pi, math.pi, D)


def test_gaussian_closed_form_at_random_angles(oracle_mod):
    from oracle import reference as ref
    g = Geometry(n=64, n_det=13, n_t=128, dt=2 / 128, det_theta=_random_angles(13, 1))
    blobs = [Blob(0.1, -0.05, 3 * g.h, 1.0), Blob(-0.2, 0.15, 3 * g.h, 0.7)]
    f = render_phantom(PhantomSpec(blobs=blobs, cutoff_r=10.0), g.n)
    s = oracle_mod.sizes(g)
    assert _rel(oracle_mod.forward(g, f), ref.discrete_gaussian_data(g, s, blobs)) < 1e-12


def test_explicit_uniform_angles_reproduce_the_arc(oracle_mod):
    g = Geometry(n=32, n_det=20, n_t=64, dt=2 / 64, arc_span=math.radians(200), arc_center=0.4)
    ge = g.with_(det_theta=tuple(g.det_angles()))
    f = np.random.default_rng(2).standard_normal((g.n, g.n))
    assert _rel(oracle_mod.forward(ge, f), oracle_mod.forward(g, f)) < 1e-13
    d = np.random.default_rng(3).standard_normal((g.n_det, g.n_t))
    assert _rel(oracle_mod.adjoint(ge, d), oracle_mod.adjoint(g, d)) < 1e-13


def test_permutation_and_union_of_arcs(oracle_mod):
    a = Geometry(n=32, n_det=9, n_t=48, dt=2 / 48, arc_span=math.radians(60), arc_center=-1.0)
    b = Geometry(n=32, n_det=7, n_t=48, dt=2 / 48, arc_span=math.radians(45), arc_center=1.8)
    th = np.concatenate([a.det_angles(), b.det_angles()])
    perm = np.random.default_rng(4).permutation(th.size)
    u = a.with_(n_det=th.size, det_theta=tuple(th[perm]))
    f = np.random.default_rng(5).standard_normal((32, 32))
    stacked = np.concatenate([oracle_mod.forward(a, f), oracle_mod.forward(b, f)])
    assert _rel(oracle_mod.forward(u, f), stacked[perm]) < 1e-13


def test_transpose_and_impulse_at_random_angles(oracle_mod):
    from oracle import reference as ref
    g = Geometry(n=40, n_det=11, n_t=80, dt=2 / 80, det_theta=_random_angles(11, 6))
    rng = np.random.default_rng(7)
    f = rng.standard_normal((g.n, g.n))
    d = rng.standard_normal((g.n_det, g.n_t))
    lhs = float(np.sum(oracle_mod.forward(g, f) * d))
    rhs = float(np.sum(f * oracle_mod.adjoint(g, d)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    s = oracle_mod.sizes(g)
    for (dd, j) in [(0, 3), (10, 70)]:
        data = np.zeros((g.n_det, g.n_t))
        data[dd, j] = 1.0
        A = oracle_mod.adjoint(g, data)
        C = ref.discrete_impulse_adjoint(g, s, dd, j)
        assert np.abs(A - C).max() < 1e-12 * np.abs(C).max()


def test_geometry_rejects_a_wrong_angle_count():
    with pytest.raises(ValueError):
        Geometry(n=32, n_det=4, n_t=8, dt=0.25, det_theta=(0.0, 1.0))
