"""The CPU oracle against its pins, and planted mistakes against the pins.

The pins themselves (and why each is independent of the oracle's formula) are
in ``oracle_pins.py``.  ``test_planted_mistakes`` compiles variants of the
oracle's C source with one plausible error each -- the plus sign printed in
Eq. (7), z0 in place of r0, a dropped term, x and y swapped, a conjugated
product, an off-by-one pixel centre, and in the Huygens sum, Eq. (5) and the 1D
forms a wrong distance, power, prefactor or sign -- and requires every variant
to fail at least one pin.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle_pins import PINS, rel_l2


@pytest.mark.parametrize("name", sorted(PINS))
def test_pin(name):
    err, bound = PINS[name]()
    assert err < bound, (name, err, bound)


def test_threads():
    assert oracle.threads() >= 1
    assert oracle.threads(3) == 3


def test_mpmath_rounding_tiny():
    """FP64 rounding of the direct sum against 50 digits (3x3 points, 4x4 pixels).

    This re-evaluates the same definition and so checks rounding only: the
    largest phase is k z0 ~ 1.2e6 rad, which FP64 forms with a relative error
    of a few ulp, so the bound is 8 * 2^-53 * k (z0 + max chirp).
    """
    rng = np.random.default_rng(7)
    x, y = synth.jittered_grid(rng, 3, 3, 8e-6, 2e-6)
    d = synth.sinusoidal_relief(x, y, 50e-6, 1e-3)
    u = synth.random_field(rng, 3, 3)
    lam, z0, p2 = 532e-9, 0.1, 8e-6
    ix, iy = np.meshgrid(np.arange(4), np.arange(4))
    ix, iy = ix.reshape(-1), iy.reshape(-1)
    k = 2 * np.pi / lam
    bound = 8 * 2.0 ** -53 * k * (z0 + 1e-3) + 1e-14
    for inc in ("plane", "none"):
        got = oracle.direct(x, y, d, u, lam, z0, p2, p2, 4, 4, ix, iy, incident=inc)
        ref = oracle.mp_direct(x, y, d, u, lam, z0, p2, p2, 4, 4, ix, iy, incident=inc)
        assert rel_l2(got, ref) < bound, (inc, rel_l2(got, ref), bound)


def test_domain_error():
    x = np.zeros(2); y = np.zeros(2); d = np.array([0.0, 0.2])
    u = np.ones(2, dtype=np.complex64)
    with pytest.raises(ValueError):
        oracle.direct(x, y, d, u, 532e-9, 0.2, 8e-6, 8e-6, 4, 4, [0], [0])


def test_subset_consistency():
    """Evaluating pixels one by one, in any order, equals evaluating a block."""
    w = synth.config("cap_2048", side=32, out=24)
    block = oracle.direct_grid(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    ix, iy = synth.sample_pixels(w.mx, w.my, 50, seed=5)
    perm = np.random.default_rng(0).permutation(len(ix))
    some = oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                         ix[perm], iy[perm], nthreads=2)
    assert np.array_equal(some, block[iy[perm], ix[perm]])


# (original text, planted mistake) pairs applied to the oracle's C source
MUTANTS = {
    "cross_term_plus": ("- (x[j] * X + y[j] * Y) / r0)", "+ (x[j] * X + y[j] * Y) / r0)"),
    "cross_term_z0": ("- (x[j] * X + y[j] * Y) / r0)", "- (x[j] * X + y[j] * Y) / z0)"),
    "source_chirp_z0": ("(x[j] * x[j] + y[j] * y[j]) / (2.0 * r0)", "(x[j] * x[j] + y[j] * y[j]) / (2.0 * z0)"),
    "dropped_minus_d": ("arg = k * (-d[j] + ", "arg = k * (0.0 + "),
    "xy_swapped": ("(x[j] * X + y[j] * Y)", "(x[j] * Y + y[j] * X)"),
    "dropped_output_chirp": ("(X * X + Y * Y) / (2.0 * z0)", "0.0"),
    "dropped_kz0": ("sincos(k * (z0 + ", "sincos(k * (0.0 + "),
    "conjugated_product": ("sr += ur * c - ui * s;", "sr += ur * c + ui * s;"),
    "centre_off_by_one": ("(double)(ix[e] - mx / 2)", "(double)(ix[e] - (mx - 1) / 2)"),
    "incident_sign": ("arg += k * d[j];", "arg -= k * d[j];"),
    "prefactor_lambda": ("1.0 / (lambda * z0)", "1.0 / (lambda * 0.1)"),
    "window_offset_sign": ("const double X = x0 + p2x * (double)(ix[e] - mx / 2);",
                           "const double X = -x0 + p2x * (double)(ix[e] - mx / 2);"),
    "window_offset_dropped": ("const double Y = y0 + p2y * (double)(iy[e] - my / 2);",
                              "const double Y = p2y * (double)(iy[e] - my / 2);"),
    # mistakes in Eq. (5) and the Huygens sum, Eq. (2)-(3)
    "eq5_output_chirp_z0": ("- (x[j] * X + y[j] * Y) / r0 + (X * X + Y * Y) / (2.0 * r0));",
                            "- (x[j] * X + y[j] * Y) / r0 + (X * X + Y * Y) / (2.0 * z0));"),
    "eq2_r_with_z0": ("sqrt(dx * dx + dy * dy + r0 * r0);", "sqrt(dx * dx + dy * dy + z0 * z0);"),
    "eq2_amplitude_1_over_r": ("amp = 1.0 / (r * r);", "amp = 1.0 / r;"),
    "eq2_prefactor_without_z0": ("a = z0 / lambda;", "a = 1.0 / lambda;"),
    "eq2_phase_sign": ("arg = k * r;", "arg = -k * r;"),
    "eq2_dx_sign": ("const double dx = X - x[j], dy = Y - y[j];", "const double dx = X + x[j], dy = Y - y[j];"),
    # mistakes in the one-dimensional forms
    "line_prefactor_2d_form": ("a = 1.0 / sqrt(lambda * z0);", "a = 1.0 / (lambda * z0);"),
    "line_no_quarter_turn": ("phase = k * (z0 + X * X / (2.0 * z0)) - pi / 4.0;",
                             "phase = k * (z0 + X * X / (2.0 * z0));"),
    "line_eq5_chirp_z0": ("+ X * X / (2.0 * r0));", "+ X * X / (2.0 * z0));"),
    "line_cross_term_plus": ("- x[j] * X / r0", "+ x[j] * X / r0"),
    "line_centre_off_by_one": ("(double)(ix[e] - m / 2)", "(double)(ix[e] - (m - 1) / 2)"),
    "line_eq2_power": ("amp = 1.0 / (rho * sqrt(rho));", "amp = 1.0 / (rho * rho);"),
    "line_eq2_rho_with_z0": ("sqrt(dx * dx + r0 * r0);", "sqrt(dx * dx + z0 * z0);"),
    "line_eq2_no_quarter_turn": ("phase = -pi / 4.0;", "phase = 0.0;"),
    # mistakes in the adjoint alone
    "adjoint_not_conjugated": ("sr += c * gr + s * gi;", "sr += c * gr - s * gi;"),
    "adjoint_prefactor_sign": ("out[2 * e] = -a * si;", "out[2 * e] = a * si;"),
    "adjoint_dropped_output_chirp": ("arg += k * (z0 + (X * X + Y * Y) / (2.0 * z0));", "arg += k * z0;"),
    "adjoint_centre_off_by_one": ("(double)(ix - mx / 2)", "(double)(ix - (mx - 1) / 2)"),
    "adjoint_swapped_axes": ("double)(iy - my / 2)", "double)(iy - mx / 2)"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle._SRC).read()
    assert src.count(old) >= 1, (name, old)
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                    str(path), "-lm"], check=True)
    return oracle.load_library(str(lib))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes(tmp_path, name):
    """Each variant must fail some pin (the pins run until the first that fails)."""
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    for pin, fn in PINS.items():
        err, bound = fn(lib=lib)
        if not err < bound:
            return
    raise AssertionError(f"planted mistake {name} passed every pin")
