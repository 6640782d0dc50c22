"""GPU parity for the destination-window offset and for accumulating several
surfaces into one destination (asf_forward_add), against the FP64 oracle."""
import os

import numpy as np
import pytest

import synth
from gpu_util import rel_l2, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-4}
ORACLE_THREADS = min(16, os.cpu_count() or 1)
X0, Y0 = 0.517e-3, -0.333e-3   # not whole pixels


def _oracle_grid(w, x0=0.0, y0=0.0, u=None):
    import oracle
    return oracle.direct_grid(w.x, w.y, w.d, w.u if u is None else u, w.lam, w.z0, w.p2x, w.p2y,
                              w.mx, w.my, incident=w.incident, nthreads=ORACLE_THREADS, x0=x0, y0=y0)


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_offset_window(fft):
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("sinusoid_128")
    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft, x0=X0, y0=Y0)
    got = plan.forward(u).cpu().numpy().astype(np.complex128)
    plan.close()
    err = rel_l2(got, _oracle_grid(w, X0, Y0))
    print(f"offset window {fft}: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


def test_two_surfaces_accumulate_into_one_destination():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    a = synth.config("sinusoid_128", side=96, out=128, seed=0)
    b = synth.config("sinusoid_128", side=80, out=128, seed=5)
    b.x = b.x + 0.31e-3          # a second surface beside the first, same optics
    b.d = synth.sinusoidal_relief(b.x, b.y, 30e-6, 0.6e-3)
    out = torch.empty((128, 128), dtype=torch.complex64, device="cuda")
    plans = []
    for i, w in enumerate((a, b)):
        x, y, d, u = to_dev(torch, w)
        plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, x0=X0, y0=Y0)
        plan.forward(u, out=out, accumulate=i > 0)
        plans.append(plan)
    got = out.cpu().numpy().astype(np.complex128)
    for plan in plans:
        plan.close()
    want = _oracle_grid(a, X0, Y0) + _oracle_grid(b, X0, Y0)
    err = rel_l2(got, want)
    print(f"two surfaces accumulated: rel-L2 {err:.3e}")
    assert err <= TOL["fp32"]


def test_adjoint_with_offset_window():
    torch = torch_gpu()
    import oracle
    import paper_1203_3583_amd as asf

    w = synth.config("sinusoid_128", side=96, out=64)
    x, y, d, _ = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, x0=X0, y0=Y0)
    g2 = synth.random_field(np.random.default_rng(3), w.mx, w.my).reshape(w.my, w.mx)
    got = plan.adjoint(torch.from_numpy(g2).cuda()).cpu().numpy().astype(np.complex128)
    plan.close()
    want = oracle.adjoint(w.x, w.y, w.d, g2, w.lam, w.z0, w.p2x, w.p2y, incident=w.incident,
                          nthreads=ORACLE_THREADS, x0=X0, y0=Y0)
    err = rel_l2(got, want)
    print(f"adjoint offset window: rel-L2 {err:.3e}")
    assert err <= TOL["fp32"]
