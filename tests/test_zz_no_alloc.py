"""The forward variant for callers that cannot allocate (asf_forward_static), called
through the C ABI: its fine grid and column-pass output live in the library's fixed
device scratch array.  Its output must equal asf_forward's on the same plan bit for
bit (the same kernels on the same data; the spread sums in integers) on two calls
in a row, the second with a smaller problem (the array keeps the first call's
contents, which the second must not read, also where the second leaves most of
the fine grid unwritten and its column pass reads those tiles as zeros), and a plan too large for the array
must be refused on the host with ASF_ESIZE."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _forward_both(torch, asf, w, fft):
    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    a = torch.empty((w.my, w.mx), dtype=torch.complex64, device="cuda")
    b = torch.full((w.my, w.mx), float("nan"), dtype=torch.complex64, device="cuda")
    lib = asf.lib()
    assert lib.asf_forward(plan._h, u.data_ptr(), a.data_ptr(), stream) == 0, asf.last_error()
    assert lib.asf_forward_static(plan._h, u.data_ptr(), b.data_ptr(), stream) == 0, asf.last_error()
    torch.cuda.synchronize()
    info = plan.info()
    unwritten = int((plan.workspace_view(info["off_live"], info["ntiles"], torch.uint8) == 0).sum())
    plan.close()
    return a.cpu().numpy(), b.cpu().numpy(), unwritten


def _clusters(out):
    """24 clusters of 1500 points, each within a tile or two of the fine grid: the
    spreading leaves most tiles unwritten, so the array's cells there keep the
    previous call's sums, which the column pass must not read."""
    rng = np.random.default_rng(31)
    centres = rng.uniform(-5e-3, 5e-3, size=(24, 2))
    x = (centres[:, 0, None] + rng.uniform(-4e-6, 4e-6, size=(24, 1500))).reshape(-1)
    y = (centres[:, 1, None] + rng.uniform(-4e-6, 4e-6, size=(24, 1500))).reshape(-1)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    u = synth.random_field(rng, 1, x.size).reshape(-1)
    return synth.Workload("clusters", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, out, out)


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_static_scratch_forward_matches_forward(fft):
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    # the largest destination the array holds; the same grid with fewer points, most of
    # its tiles left unwritten; a smaller grid with another surface
    for w in (synth.config("cap_2048", side=1024, out=1024), _clusters(1024),
              synth.config("sinusoid_128", side=96, out=64)):
        ref, got, unwritten = _forward_both(torch, asf, w, fft)
        print(f"{w.name} {w.mx}x{w.my} {fft}: identical {np.array_equal(ref, got)}, "
              f"{unwritten} tiles unwritten")
        assert np.all(np.isfinite(got))
        assert np.array_equal(ref, got)
        if w.name == "clusters":
            assert unwritten > 1000


def test_static_scratch_refuses_a_plan_too_large():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("cap_2048", side=64, out=2048)       # 4096^2 fine grid: 192 MiB > 48 MiB
    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    out = torch.empty((w.my, w.mx), dtype=torch.complex64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = asf.lib().asf_forward_static(plan._h, u.data_ptr(), out.data_ptr(), stream)
    plan.close()
    assert rc == asf.asf.ASF_ESIZE
    assert "static scratch" in asf.last_error()
