"""Planted mistakes in the oracle are caught by its pins.

Each mutant is a copy of oracle/pat_oracle.c with one plausible slip (a dropped
weight, a flipped sign, a swapped axis, an off-by-one grid).  It is compiled on
the CPU into a temporary library and the pins of test_oracle_pins.py are run
against it; at least one pin must fail for every mutant.
"""
import os

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "pat_oracle.c")

MUTANTS = {
    "drop_W_lambda": ("return lam_at(s, n) * s->dlam / (2.0 * PI);", "return s->dlam / (2.0 * PI);"),
    "swap_x_y": ("double kx = lam * cos(psi), ky = lam * sin(psi);\n            for (int j = 0; j < N; ++j) { cx[j] = cos(kx",
                 "double kx = lam * sin(psi), ky = lam * cos(psi);\n            for (int j = 0; j < N; ++j) { cx[j] = cos(kx"),
    "fourier_sign": ("re += cy * a - sy * b;\n                im -= sy * a + cy * b;",
                     "re += cy * a + sy * b;\n                im += sy * a - cy * b;"),
    "time_grid_from_zero": ("return j * g->dt;", "return (j - 1) * g->dt;"),
    "detector_no_half_offset": ("(d + 0.5) * g->arc_span", "d * g->arc_span"),
    "kappa_sign": ("s->dlam * s->dlam / (24.0 * PI)", "-s->dlam * s->dlam / (24.0 * PI)"),
    "drop_angular_normalisation": ("P[q] = acc / NP;", "P[q] = acc;"),
    "detector_phase_sign": ("cos(th - psi_at(&s, l))", "cos(th + psi_at(&s, l))"),
    "adjoint_phase_sign": ("im -= qv * sin(ph);", "im += qv * sin(ph);"),
    "pixel_no_half_offset": ("(k + 0.5) * (2.0 / g->n)", "(k + 0.0) * (2.0 / g->n)"),
    "sine_propagator": ("acc += W_at(&s, n) * cos(", "acc += W_at(&s, n) * sin("),
    "n_lam_off_by_one": ("/ h + 1e-9);", "/ h + 1e-9) - 1;"),
    "K_rule_too_small": ("z + 10.0 * cbrt(z) - 1e-9", "z + 1.0 * cbrt(z) - 1e-9"),
    "adjoint_drops_kappa": ("h * h * v + s.kappa * h * h * data_sum", "h * h * v"),
}

CHECKS = [
    lambda: pins.test_sizes_by_hand(oracle, 2, dict(M=1024, n_lam=512, K=476, n_psi=972)),
    lambda: pins.test_dot_product_adjoint(oracle),
    lambda: pins.test_gaussian_closed_form_forward(oracle),
    lambda: pins.test_impulse_closed_form_adjoint(oracle),
    lambda: pins.test_polar_rays_equal_numpy_fft(oracle),
    lambda: pins.test_mode_form_equals_plane_wave_form(oracle),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new, 1)
    msrc = tmp_path / ("mutant_%s.c" % name)
    msrc.write_text(mutated)
    lib = oracle.compile_source(str(msrc), str(tmp_path / ("libmutant_%s.so" % name)))
    handle = oracle.use_library(lib)
    caught = []
    try:
        for i, chk in enumerate(CHECKS):
            try:
                chk()
            except (AssertionError, ValueError):
                caught.append(i)
    finally:
        oracle.restore_library(handle)
    assert caught, "mutant %s passed every pin" % name


def test_unmutated_source_passes_all_checks():
    oracle.build(force=False)
    for chk in CHECKS:
        chk()
