"""GPU parity of the adjoint g1 = A^H g2 (the type-2 direction) against the FP64
CPU oracle's direct sum, element by element over source points, plus the GPU
forward/adjoint pair against the inner-product identity <A u, g> = <u, A^H g>.
Bars as for the forward: relative L2 <= 1e-5 with FP32 FFT stages, <= 1e-4 with
split-FP16 FFT stages."""
import os

import numpy as np
import pytest

import synth
from gpu_util import rel_l2, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-4}
ORACLE_THREADS = min(16, os.cpu_count() or 1)


def _g2(w, seed=21):
    rng = np.random.default_rng(seed)
    return synth.random_field(rng, w.mx, w.my).reshape(w.my, w.mx)


def _gpu_adjoint(w, g2, fft="fp32"):
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    x, y, d, _ = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft,
                    incident=w.incident)
    g1 = plan.adjoint(torch.from_numpy(np.ascontiguousarray(g2)).cuda())
    torch.cuda.synchronize()
    plan.close()
    return g1.cpu().numpy().astype(np.complex128)


def _oracle_adjoint(w, g2, jidx=None):
    import oracle
    return oracle.adjoint(w.x, w.y, w.d, g2, w.lam, w.z0, w.p2x, w.p2y, jidx, incident=w.incident,
                          nthreads=ORACLE_THREADS)


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_adjoint_sinusoid_128_all_points(fft):
    w = synth.config("sinusoid_128")
    g2 = _g2(w)
    got = _gpu_adjoint(w, g2, fft)
    want = _oracle_adjoint(w, g2)
    err = rel_l2(got, want)
    print(f"adjoint sinusoid_128 {fft}: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_adjoint_ragged_nonsquare_no_incident(fft):
    rng = np.random.default_rng(8)
    x, y = synth.jittered_grid(rng, 77, 53, 8e-6, 2.4e-6)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    u = synth.random_field(rng, 77, 53)
    w = synth.Workload("ragged", x, y, d, u, 532e-9, 0.1, 8e-6, 6e-6, 128, 64, 1e-5, "none")
    g2 = _g2(w, seed=3)
    err = rel_l2(_gpu_adjoint(w, g2, fft), _oracle_adjoint(w, g2))
    print(f"adjoint ragged {fft}: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
@pytest.mark.parametrize("mx,my", [(16, 2048), (2048, 16), (32, 1024), (1024, 32), (64, 512), (512, 64),
                                   (16, 4096), (4096, 16)])
def test_adjoint_every_transform_length(mx, my, fft):
    """The adjoint's passes and interpolation at fine-grid lengths 32 .. 8192 along each
    axis (32-cell sides wrap a tile's region onto itself), 2999 scattered points whose
    frequencies wrap: every point against the oracle."""
    rng = np.random.default_rng(mx * 5 + my)
    n = 2999
    x = rng.uniform(-5e-4, 5e-4, n)
    y = rng.uniform(-5e-4, 5e-4, n)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    u = np.zeros(n, dtype=np.complex64)
    w = synth.Workload("lengths", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, mx, my, 1e-5, "plane")
    g2 = _g2(w, seed=mx + my)
    err = rel_l2(_gpu_adjoint(w, g2, fft), _oracle_adjoint(w, g2))
    print(f"adjoint {mx} x {my} {fft}: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
def test_adjoint_every_width(tol):
    """Interpolation at every spreading width the tolerances select (3 .. 9): the
    requested accuracy, or the FP32 bar of 1e-5 below it."""
    rng = np.random.default_rng(12)
    x, y = synth.jittered_grid(rng, 64, 64, 8e-6, 2e-6)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    u = synth.random_field(rng, 64, 64)
    w = synth.Workload("width", x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 64, 64, tol, "plane")
    g2 = _g2(w, seed=6)
    err = rel_l2(_gpu_adjoint(w, g2), _oracle_adjoint(w, g2))
    print(f"adjoint tol {tol}: rel-L2 {err:.3e}")
    assert err <= max(tol, 1e-5)


def test_adjoint_wrapping_frequencies():
    # destination pitch large enough that p2 xi spans more than one period
    rng = np.random.default_rng(9)
    x, y = synth.jittered_grid(rng, 64, 64, 8e-6, 2.4e-6)
    d = synth.sinusoidal_relief(x, y, 30e-6, 0.5e-3)
    u = synth.random_field(rng, 64, 64)
    w = synth.Workload("wrap", x, y, d, u, 532e-9, 0.1, 80e-6, 70e-6, 64, 64, 1e-5, "plane")
    g2 = _g2(w, seed=4)
    err = rel_l2(_gpu_adjoint(w, g2), _oracle_adjoint(w, g2))
    print(f"adjoint wrapping: rel-L2 {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_adjoint_cap_2048_full_size_sampled(fft):
    w = synth.config("cap_2048")
    g2 = _g2(w, seed=5)
    got = _gpu_adjoint(w, g2, fft)
    rng = np.random.default_rng(6)
    jidx = rng.choice(w.n, 192, replace=False)
    want = _oracle_adjoint(w, g2, jidx)
    err = rel_l2(got[jidx], want)
    print(f"adjoint cap_2048 {fft}: rel-L2 {err:.3e} on {len(jidx)} points")
    assert err <= TOL[fft]


@pytest.mark.parametrize("name,kw", [("sinusoid_128", {}), ("cap_2048", {"side": 256})])
def test_inner_product_identity(name, kw):
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config(name, **kw)
    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol)
    g = torch.from_numpy(_g2(w, seed=7)).cuda()
    au = plan.forward(u).cpu().numpy().astype(np.complex128)
    ahg = plan.adjoint(g).cpu().numpy().astype(np.complex128)
    ahg2 = plan.adjoint(g).cpu().numpy()
    plan.close()
    lhs = np.vdot(g.cpu().numpy().astype(np.complex128).reshape(-1), au.reshape(-1))
    rhs = np.vdot(ahg, w.u.astype(np.complex128))
    scale = np.linalg.norm(au) * np.linalg.norm(g.cpu().numpy())
    print(f"{name}: |<Au,g> - <u,A^H g>| / (|Au| |g|) = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) / scale <= 1e-6
    # interpolation has no atomics: a repeat is bitwise identical
    assert np.array_equal(ahg2, ahg.astype(np.complex64))
