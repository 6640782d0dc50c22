"""GPU parity on coherent and high-dynamic-range sources.

Both block-scaled stages have an error floor set by the largest value of their
block: the fixed-point spread rounds every term to 2^-22 of its tile's largest
|Re c|, |Im c|, and the split-FP16 FFT scales each workgroup's transforms by a
power of two from their largest entry.  Random-phase sources spread energy
evenly; these cases do not:

* the zero-phase unit source on the differentiation configuration's spherical
  cap (R = 80 mm, 1024^2 at 8 um, lambda = 532 nm, z0 = 0.15 m) -- the start of
  its phase descent -- at full size, on a centre crop, a corner crop and random
  pixels;
* one bright point over a field 10^4 times weaker: the whole output, and the weak
  field's own image recovered by linearity (the output minus the bright point's
  output) against the oracle's image of the weak field alone.

Bars: relative L2 1e-5 (FP32 FFT) and 1e-4 (split-FP16) on the fields
themselves.  The weak image is 1.5e-2 of the whole output's norm, so an error of
the whole at the bar is 1e-5 / 1.5e-2 ~ 7e-4 of it (FP32) and ~7e-3 (split);
those are its bars.
"""
import os

import numpy as np
import pytest

import synth
from gpu_util import gpu_forward, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-4}
THREADS = min(16, os.cpu_count() or 1)


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_zero_phase_unit_source_on_cap(fft):
    import oracle

    w = synth.config("holo_1024")          # u1 = 1: zero phase, unit amplitude
    assert np.all(w.u == 1)
    got, _ = gpu_forward(w, fft)
    args = (w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    c = 128
    sets = {
        "centre": (range(w.mx // 2 - c // 2, w.mx // 2 + c // 2), range(w.my // 2 - c // 2, w.my // 2 + c // 2)),
        "corner": (range(w.mx - c, w.mx), range(w.my - c, w.my)),
    }
    for name, (rx, ry) in sets.items():
        want = oracle.crop_gemm(*args, rx, ry, incident=w.incident, nthreads=THREADS)
        err = rel_l2(got[np.ix_(list(ry), list(rx))], want)
        print(f"zero-phase cap {fft} {name} {c}^2: rel-L2 {err:.3e}")
        assert err <= TOL[fft], name
    ix, iy = synth.sample_pixels(w.mx, w.my, 1024, seed=1)
    want = oracle.direct(*args, ix, iy, incident=w.incident, nthreads=THREADS)
    err = rel_l2(got[iy, ix], want)
    print(f"zero-phase cap {fft} random 1024: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_bright_point_over_weak_field(fft):
    import dataclasses

    import oracle

    base = synth.config("cap_2048", side=256, out=256)
    rng = np.random.default_rng(17)
    weak = (1e-4 * synth.random_field(rng, 256, 256)).astype(np.complex64)
    j = 256 * 131 + 97                      # one point near the centre
    point = np.zeros_like(weak)
    point[j] = 1.0
    total = weak.copy()
    total[j] += 1.0                         # the bright point on top of the weak field
    runs = {}
    for name, u in (("total", total), ("point", point), ("weak", weak)):
        wl = dataclasses.replace(base, name=name, u=u)
        got, _ = gpu_forward(wl, fft)
        want = oracle.crop_gemm(wl.x, wl.y, wl.d, wl.u, wl.lam, wl.z0, wl.p2x, wl.p2y, wl.mx, wl.my,
                                range(wl.mx), range(wl.my), incident=wl.incident, nthreads=THREADS)
        runs[name] = (got, want)
    ratio = np.linalg.norm(runs["weak"][1]) / np.linalg.norm(runs["total"][1])
    err_total = rel_l2(*runs["total"])
    # the weak field's image, recovered from the two GPU outputs by linearity
    err_weak = rel_l2(runs["total"][0] - runs["point"][0], runs["weak"][1])
    err_weak_alone = rel_l2(*runs["weak"])
    err_point = rel_l2(*runs["point"])
    # the GPU map's own departure from linearity (no oracle involved)
    nonlin = rel_l2(runs["total"][0] - runs["point"][0], runs["weak"][0])
    print(f"bright point {fft}: weak/total norm {ratio:.2e}; total {err_total:.3e}, "
          f"weak recovered {err_weak:.3e}, weak alone {err_weak_alone:.3e}, point alone {err_point:.3e}, "
          f"GPU nonlinearity / weak {nonlin:.3e}")
    assert 1e-2 < ratio < 2e-2
    assert err_total <= TOL[fft]
    assert err_weak_alone <= TOL[fft]
    assert err_weak <= TOL[fft] / 1.5e-2
