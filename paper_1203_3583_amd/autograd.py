"""Differentiable forward for PyTorch: gradients through the adjoint transform.

``propagate(plan, u1)`` returns u2 = A u1 (the forward of the C ABI) as a node of
the autograd graph; its backward is the adjoint g1 = A^H g2 (``asf_adjoint``),
which is PyTorch's rule for a complex linear map (the gradient of u1 is A^H
times the gradient of u2).  Both directions run the HIP kernels; the plan's
geometry (x1, y1, d1) is a constant of the graph.

``intensity_loss`` and ``phase_descent`` build the phase-hologram problem on a
curved surface: a phase-only source u1 = a exp(i theta) on the plan's surface and
the loss || |u2|^2 - T ||^2 against a target intensity T.
"""
from __future__ import annotations


def _torch():
    import torch

    return torch


class _Propagate:
    """Holder of the autograd.Function (built lazily so importing needs no torch)."""

    fn = None

    @classmethod
    def get(cls):
        if cls.fn is None:
            torch = _torch()

            class Propagate(torch.autograd.Function):
                @staticmethod
                def forward(ctx, u1, plan):
                    ctx.plan = plan
                    return plan.forward(u1.contiguous())

                @staticmethod
                def backward(ctx, grad_u2):
                    g = grad_u2
                    if g.dtype != torch.complex64:
                        g = g.to(torch.complex64)
                    return ctx.plan.adjoint(g.contiguous()), None

            cls.fn = Propagate
        return cls.fn


def propagate(plan, u1):
    """u2 = A u1 (complex64 [my, mx]) with autograd support through the adjoint."""
    return _Propagate.get().apply(u1, plan)


def intensity_loss(plan, theta, amp, target):
    """|| |A (amp exp(i theta))|^2 - target ||^2 / || target ||^2 (float64 scalar).

    theta, amp: real [n] tensors on the plan's device (theta may require grad);
    target: real [my, mx] tensor in the units of |u2|^2 (see ``energy_matched``).
    """
    torch = _torch()
    u1 = torch.polar(amp.to(torch.float32), theta.to(torch.float32))
    u2 = propagate(plan, u1)
    inten = (u2.real.double() ** 2 + u2.imag.double() ** 2)
    t = target.double()
    return ((inten - t) ** 2).sum() / (t * t).sum()


def energy_matched(plan, amp, target, theta=None):
    """target rescaled so that its sum equals the energy sum |u2|^2 over the destination
    window of the source amp exp(i theta) (default theta = 0).  The window's energy
    depends on theta (the window is finite), so a caller fixes this scale once per
    problem and uses the same target for every iteration and every start it compares."""
    torch = _torch()
    th = torch.zeros_like(amp) if theta is None else theta
    with torch.no_grad():
        u2 = plan.forward(torch.polar(amp.to(torch.float32), th.to(torch.float32)).contiguous())
        e = float((u2.real.double() ** 2 + u2.imag.double() ** 2).sum())
    t = target.double()
    return t * (e / float(t.sum()))


def phase_descent(plan, amp, target, steps=50, lr=0.05, theta0=None, callback=None):
    """Adam on the source phase theta for ``intensity_loss`` against ``target`` as given
    (in units of |u2|^2: an intensity the forward method produced, or a target scaled
    once with ``energy_matched``), from theta0 (default zero phase).  Returns
    (theta, losses); descents from different starts against the same target are
    comparable loss for loss."""
    torch = _torch()
    theta = (torch.zeros_like(amp, dtype=torch.float64) if theta0 is None
             else theta0.detach().to(torch.float64).clone())
    target = target.double()
    theta.requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=lr)
    losses = []
    for it in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = intensity_loss(plan, theta, amp, target)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        if callback is not None:
            callback(it, losses[-1])
    return theta.detach(), losses
