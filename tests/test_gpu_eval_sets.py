"""GPU parity on the full-size configurations' evaluation sets.

The 2048^2 spherical cap and the 4096^2 sinusoidal relief run at full size
through the C ABI in both FFT precisions.  Each output is compared element by
element with the FP64 oracle on three sets, each at its own bar: a 256^2 centre
crop, a 256^2 corner crop (largest |m|, |n|) and 4096 random pixels.  The
oracle's values were written by ``tests/golden/make_eval_sets.py`` (which runs
``oracle.crop_gemm`` and ``oracle.direct`` only); the test first checks that
they were computed from exactly the inputs ``synth`` generates now.
"""
import importlib.util
import os

import numpy as np
import pytest

import synth
from gpu_util import gpu_forward, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-4}
HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    spec = importlib.util.spec_from_file_location("make_eval_sets", os.path.join(HERE, "golden", "make_eval_sets.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
@pytest.mark.parametrize("name", ["cap_2048", "sinusoid_4096"])
def test_full_size_eval_sets(name, fft):
    g = golden()
    w = synth.config(name)
    sets, digest = g.load(name)
    assert digest == g.input_digest(w), "stored oracle values were computed from other inputs"
    got, info = gpu_forward(w, fft)
    errs = {}
    for s, (ix, iy, want) in sets.items():
        errs[s] = rel_l2(got[iy, ix], want)
        print(f"{name} {fft} {s} ({len(ix)} pixels): rel-L2 {errs[s]:.3e}")
    for s, e in errs.items():
        assert e <= TOL[fft], (s, e)
