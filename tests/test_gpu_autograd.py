"""Gradients through the GPU path: autograd of the phase-hologram loss, whose
backward is the adjoint kernel, against the FP64 gradient from the oracle (itself
pinned by finite differences in test_gradient_pin.py), and a short phase descent
on the curved-surface hologram problem."""
import numpy as np
import pytest

import synth
from gpu_util import to_dev, torch_gpu
from test_gradient_pin import grad_fp64, problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fft,bar", [("fp32", 2e-5), ("split_fp16", 2e-4)])
def test_autograd_matches_oracle_gradient(fft, bar):
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w, theta, t = problem(side=64, seed=2)
    x, y, d, _ = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft)
    th = torch.from_numpy(theta).cuda().requires_grad_(True)
    amp = torch.ones(w.n, dtype=torch.float64, device="cuda")
    loss = asf.intensity_loss(plan, th, amp, torch.from_numpy(t).cuda())
    loss.backward()
    got = th.grad.cpu().numpy()
    plan.close()
    want = grad_fp64(w, theta, t)
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"autograd {fft}: rel-L2 of dL/dtheta vs FP64 oracle {err:.3e}")
    # forward and adjoint each carry ~1e-6; the loss is quartic in u2
    assert err <= bar


def test_propagate_is_linear_map_with_adjoint_backward():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("sinusoid_128", side=48, out=32)
    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    u1 = u.clone().requires_grad_(True)
    u2 = asf.propagate(plan, u1)
    g = torch.randn(w.my, w.mx, dtype=torch.complex64, device="cuda")
    (u2 * g.conj()).real.sum().backward()
    # d Re<g, A u> / d conj(u) convention: the gradient is A^H g
    want = plan.adjoint(g.contiguous())
    torch.cuda.synchronize()
    assert torch.allclose(u1.grad, want, rtol=0, atol=1e-6 * float(want.abs().max()))
    plan.close()


def test_phase_descent_lowers_the_loss():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("holo_1024", side=256)
    x, y, d, _ = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft="split_fp16")
    amp = torch.ones(w.n, dtype=torch.float64, device="cuda")
    target = asf.energy_matched(plan, amp, torch.from_numpy(w.meta["target"]).cuda())
    _, losses = asf.phase_descent(plan, amp, target, steps=40, lr=0.1)
    plan.close()
    print("phase descent losses:", " ".join(f"{v:.4f}" for v in losses[::5]), f"final {losses[-1]:.4f}")
    assert losses[-1] < 0.1 * losses[0]


@pytest.mark.parametrize("fft,bar", [("fp32", 2e-5), ("split_fp16", 2e-4)])
def test_full_size_descent_and_sampled_gradient(fft, bar):
    """The differentiation configuration at its stated size: 1024^2 phase-only source
    on the R = 80 mm cap, target from Gaussian-filtered noise (scaled once to the
    zero-phase window energy).  The first gradient, dL/dtheta_j = -4 Im(u1_j
    conj(g_j)) / ||T||^2 with g = A^H ((|u2|^2 - T) u2), is checked at 256 sampled
    points against the oracle's adjoint of the residual the GPU forward produced (the
    forward itself is checked on this source in test_gpu_dynamic_range); then 30
    Adam steps must lower the loss."""
    torch = torch_gpu()
    import oracle
    import paper_1203_3583_amd as asf

    w = synth.config("holo_1024")
    x, y, d, _ = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft)
    amp = torch.ones(w.n, dtype=torch.float64, device="cuda")
    target = asf.energy_matched(plan, amp, torch.from_numpy(w.meta["target"]).cuda())
    th = torch.zeros(w.n, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = asf.intensity_loss(plan, th, amp, target)
    loss.backward()
    got = th.grad.cpu().numpy()
    u2 = plan.forward(torch.ones(w.n, dtype=torch.complex64, device="cuda")).cpu().numpy().astype(np.complex128)
    t = target.cpu().numpy()
    resid = (np.abs(u2) ** 2 - t) * u2
    jidx = np.sort(np.random.default_rng(4).choice(w.n, 256, replace=False))
    g = oracle.adjoint(w.x, w.y, w.d, resid, w.lam, w.z0, w.p2x, w.p2y, jidx=jidx, incident=w.incident,
                       nthreads=min(16, __import__("os").cpu_count() or 1))
    want = -4.0 * np.imag(np.conj(g)) / np.sum(t * t)     # u1 = 1
    err = float(np.linalg.norm(got[jidx] - want) / np.linalg.norm(want))
    print(f"1024^2 {fft}: sampled dL/dtheta vs oracle adjoint rel-L2 {err:.3e}")
    assert err <= bar
    _, losses = asf.phase_descent(plan, amp, target, steps=30, lr=0.1)
    plan.close()
    print(f"1024^2 {fft} descent:", " ".join(f"{v:.4f}" for v in losses[::5]), f"final {losses[-1]:.4f}")
    assert losses[-1] < 0.3 * losses[0]
