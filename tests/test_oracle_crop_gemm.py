"""The oracle's second implementation, ``crop_gemm`` (Eq. (7) as FP64 matrix
products over a rectangle of pixels), against its pins.

* It must reproduce ``direct`` (the plain per-term sum) on the whole 128^2
  sinusoidal relief and on a 512^2 spherical cap whose frequencies wrap.
* It must pass, on its own, the closed-form pins that ``direct`` passes: the
  centred DFT of a flat uniform grid, the textbook Gaussian beams (tilted,
  anisotropic, raised and lowered, two heights, off-axis window), the separable
  matrix form and the single-point magnitude.  These do not depend on either
  implementation's arithmetic.
* Planted mistakes in its source (the cross term's sign or 1/r0, the axes of
  the two factors, the plane-wave term, the post-phase) must each fail a pin.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle
import synth
from oracle_pins import PINS, rel_l2

GRID_PINS = ["centred_dft_flat_none", "centred_dft_raised_none", "centred_dft_raised_plane",
             "separable", "single_point", "gaussian_on_axis", "gaussian_tilted_raised",
             "gaussian_tilted_lowered", "two_heights", "window_offset_gaussian"]


def _grid_via(fn):
    """A stand-in for ``oracle.direct_grid`` that evaluates through ``fn`` (crop_gemm or a variant)."""
    def direct_grid(x, y, d, u, lam, z0, p2x, p2y, mx, my, ix_range=None, iy_range=None,
                    incident="plane", nthreads=0, lib=None, x0=0.0, y0=0.0):
        assert lib is None
        ixs = range(mx) if ix_range is None else ix_range
        iys = range(my) if iy_range is None else iy_range
        return fn(x, y, d, u, lam, z0, p2x, p2y, mx, my, ixs, iys, incident=incident, x0=x0, y0=y0)
    return direct_grid


def test_matches_direct_full_128():
    """The whole 128^2 relief: the two implementations agree to FP64 rounding (<= 1e-12)."""
    w = synth.config("sinusoid_128")
    a = oracle.direct_grid(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    b = oracle.crop_gemm(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                         range(w.mx), range(w.my))
    err = rel_l2(b, a)
    print(f"crop_gemm vs direct, 128^2 relief: {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("incident", ["plane", "none"])
def test_matches_direct_reduced_cap(incident):
    """A 512^2 spherical cap (R = 50 mm, the 2048^2 cap's optics: its frequencies wrap),
    a corner crop and a window off the axis: agreement to FP64 rounding of phases
    up to ~1e4 rad (a few 1e-12 rad per term), bound 1e-12 relative."""
    w = synth.config("cap_2048", side=512, out=512)
    ix, iy = range(512 - 40, 512), range(0, 24)
    for x0, y0 in ((0.0, 0.0), (0.31e-3, -0.17e-3)):
        a = oracle.direct_grid(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                               incident=incident, x0=x0, y0=y0)
        b = oracle.crop_gemm(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                             incident=incident, x0=x0, y0=y0, chunk=4096)
        err = rel_l2(b, a)
        print(f"crop_gemm vs direct, 512^2 cap {incident} window ({x0}, {y0}): {err:.2e}")
        assert err <= 1e-12


def test_chunking_and_threads_do_not_change_the_sum():
    w = synth.config("cap_2048", side=64, out=64)
    args = (w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, range(10, 30), range(40, 52))
    a = oracle.crop_gemm(*args, chunk=4096, nthreads=1)
    b = oracle.crop_gemm(*args, chunk=333, nthreads=3)
    assert rel_l2(b, a) <= 1e-14


def test_domain_error():
    x = np.zeros(2); y = np.zeros(2); d = np.array([0.0, 0.2])
    u = np.ones(2, dtype=np.complex64)
    with pytest.raises(ValueError):
        oracle.crop_gemm(x, y, d, u, 532e-9, 0.2, 8e-6, 8e-6, 4, 4, range(4), range(4))


@pytest.mark.parametrize("name", GRID_PINS)
def test_closed_form_pins(name, monkeypatch):
    import oracle_pins

    monkeypatch.setattr(oracle_pins.oracle, "direct_grid", _grid_via(oracle.crop_gemm))
    err, bound = PINS[name]()
    print(f"crop_gemm pin {name}: {err:.2e} (bound {bound:g})")
    assert err < bound


# (original text, planted mistake) pairs applied to crop_gemm's source
MUTANTS = {
    "cross_term_plus": ("ax = np.exp(-1j * k", "ax = np.exp(1j * k"),
    "cross_term_z0": ("(np.outer(xj, X) / r0[:, None])", "(np.outer(xj, X) / z0)"),
    "axes_swapped": ("np.outer(xj, X)", "np.outer(yj, X)"),
    "source_chirp_z0": ("(xj * xj + yj * yj) / (2.0 * r0)", "(xj * xj + yj * yj) / (2.0 * z0)"),
    "plane_term_dropped": ("arg = arg + k * dj", "arg = arg"),
    "output_chirp_dropped": ("(X[None, :] ** 2 + Y[:, None] ** 2) / (2.0 * z0)", "0.0"),
    "conjugated_factor": ("return (ay * c[:, None]).T @ ax", "return (ay * np.conj(c)[:, None]).T @ ax"),
    "centre_off_by_one": ("(ixs - mx // 2)", "(ixs - (mx - 1) // 2)"),
}


def _mutant(old, new):
    src = textwrap.dedent(inspect.getsource(oracle.crop_gemm))
    assert src.count(old) >= 1, old
    ns = {"np": np, "threads": oracle.threads}
    exec(compile(src.replace(old, new), "<crop_gemm mutant>", "exec"), ns)
    return ns["crop_gemm"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes(name, monkeypatch):
    import oracle_pins

    fn = _mutant(*MUTANTS[name])
    monkeypatch.setattr(oracle_pins.oracle, "direct_grid", _grid_via(fn))
    for pin in GRID_PINS:
        err, bound = PINS[pin]()
        if not err < bound:
            return
    raise AssertionError(f"planted mistake {name} passed every pin")
