"""Shared helpers of the GPU tests: run the HIP path on a synthetic workload and
compare it element by element with the CPU oracle."""
import numpy as np
import pytest


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, w, device="cuda:0"):
    x = torch.from_numpy(np.ascontiguousarray(w.x)).to(device)
    y = torch.from_numpy(np.ascontiguousarray(w.y)).to(device)
    d = torch.from_numpy(np.ascontiguousarray(w.d)).to(device)
    u = torch.from_numpy(np.ascontiguousarray(w.u)).to(device)
    return x, y, d, u


def gpu_forward(w, fft="fp32", tol=None, device="cuda:0"):
    """(u2 as complex128 numpy [my, mx], plan info) for workload w on the GPU."""
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    x, y, d, u = to_dev(torch, w, device)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                    tol=w.tol if tol is None else tol, fft=fft, incident=w.incident)
    out = plan.forward(u)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return out.cpu().numpy().astype(np.complex128), info


def oracle_at(w, ix, iy):
    import oracle
    return oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                         incident=w.incident)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def eval_sets(w, n_random=512, crop=32, seed=1):
    """Evaluation sets: centre crop, corner crop (largest |m|, |n|) and random pixels."""
    c0x, c0y = w.mx // 2 - crop // 2, w.my // 2 - crop // 2
    gx, gy = np.meshgrid(np.arange(c0x, c0x + crop), np.arange(c0y, c0y + crop))
    centre = (gx.reshape(-1), gy.reshape(-1))
    gx, gy = np.meshgrid(np.arange(w.mx - crop, w.mx), np.arange(w.my - crop, w.my))
    corner = (gx.reshape(-1), gy.reshape(-1))
    import synth
    rand = synth.sample_pixels(w.mx, w.my, n_random, seed=seed)
    return {"centre": centre, "corner": corner, "random": rand}
