"""The spreading kernel's polynomial table (paper_1203_3583_amd/csrc/es_poly.h) is
current with its generator and close to the exponential-of-semicircle kernel it
replaces.  Host logic only; the end-to-end accuracy is covered by the GPU tests."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_1203_3583_amd", "csrc", "gen_es_poly.py")


@pytest.fixture(scope="module")
def gen():
    spec = importlib.util.spec_from_file_location("gen_es_poly", GEN)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_header_is_current(gen):
    with open(gen.HEADER) as fh:
        assert fh.read() == gen.render()


@pytest.mark.parametrize("w,bound", [(5, 1e-5), (6, 1e-6), (7, 2e-7), (8, 2e-7), (9, 2e-7)])
def test_fp32_evaluation_error(gen, w, bound):
    # the error of the even/odd FP32 Horner evaluation the kernel performs, against psi in FP64,
    # well below the NUFFT error the width w is chosen for (10^-(w-2))
    assert gen.max_error(w) <= bound


def test_mirror_symmetry_and_peak(gen):
    w = 7
    f = np.linspace(-0.5, 0.5, 101)
    # psi_{w-1-i}(f) = psi_i(-f), which is what lets the kernel share even/odd parts
    for i in range(w):
        assert np.allclose(gen.psi_i(f, w - 1 - i, w), gen.psi_i(-f, i, w), rtol=0, atol=1e-15)
    # at f = 0 the middle cell is the kernel's peak, psi(0) = 1
    assert gen.psi_i(np.array([0.0]), 3, w)[0] == pytest.approx(1.0, abs=1e-15)
