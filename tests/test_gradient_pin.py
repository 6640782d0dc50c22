"""The phase-hologram gradient in FP64 from the oracle, pinned by finite differences.

For a phase-only source u1 = exp(i theta) and L = || |A u1|^2 - T ||^2 / ||T||^2,
  dL/dtheta_j = -4 Im(u1_j conj(g_j)) / ||T||^2,  g = A^H ((|u2|^2 - T) u2),
which uses the oracle's forward and adjoint (both pinned in test_oracle_pins).
Central differences of L computed with the FP64 forward alone must agree; this is
the reference the GPU autograd test compares with.  CPU only."""
import numpy as np

import oracle
import synth


def loss_fp64(w, theta, target):
    u1 = np.exp(1j * theta)
    u2 = oracle.direct_grid(w.x, w.y, w.d, u1, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    e = np.abs(u2) ** 2 - target
    return float(np.sum(e * e) / np.sum(target * target)), u1, u2, e


def grad_fp64(w, theta, target):
    _, u1, u2, e = loss_fp64(w, theta, target)
    g = oracle.adjoint(w.x, w.y, w.d, e * u2, w.lam, w.z0, w.p2x, w.p2y)
    return -4.0 * np.imag(u1 * np.conj(g)) / np.sum(target * target)


def problem(side=32, seed=0):
    w = synth.config("holo_1024", side=side, seed=seed)
    rng = np.random.default_rng(seed + 1)
    theta = rng.uniform(0, 2 * np.pi, w.n)
    _, _, u2, _ = loss_fp64(w, theta, np.zeros((w.my, w.mx)) + 1.0)
    t = w.meta["target"] * (np.sum(np.abs(u2) ** 2) / np.sum(w.meta["target"]))
    return w, theta, t


def test_gradient_matches_central_differences():
    """64 x 64 source and destination (the differentiation configuration's check size)."""
    w, theta, t = problem(side=64)
    g = grad_fp64(w, theta, t)
    rng = np.random.default_rng(3)
    h = 1e-5
    for j in rng.choice(w.n, 6, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (loss_fp64(w, tp, t)[0] - loss_fp64(w, tm, t)[0]) / (2 * h)
        # central difference: O(h^2) truncation plus FP64 rounding of L / h (~1e-10 here)
        assert abs(fd - g[j]) <= 1e-8 * np.max(np.abs(g)), (j, fd, g[j])


def test_gradient_vanishes_at_target():
    # if the target is the field's own intensity, every phase is stationary
    w, theta, _ = problem(side=16)
    u2 = oracle.direct_grid(w.x, w.y, w.d, np.exp(1j * theta), w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    g = grad_fp64(w, theta, np.abs(u2) ** 2)
    assert np.max(np.abs(g)) < 1e-9
