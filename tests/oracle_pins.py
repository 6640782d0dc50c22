"""Pins of the CPU oracle against results the mathematics fixes on its own.

Each pin reduces Eq. (7) (Sec. 2) to a case whose answer does not come from
re-typing the oracle's formula, and returns (error, bound):

* ``centred_dft_*``: a uniform source grid at constant height with the matching
  destination pitch p2 = lambda r0 / (N p1) turns the sum into a centred DFT
  (numpy.fft) -- pins the cross term's sign, its 1/r0 scaling, the pixel
  centring and the axis assignment;
* ``gaussian_*``: a sampled Gaussian source turns the sum (times the cell area)
  into a Riemann sum of the Fresnel integral, whose value is the textbook
  paraxial Gaussian beam (waist, radius of curvature, Gouy phase) -- pins the
  prefactor, the output chirp, the source chirp with r0 = z0 - d1 and the
  -k d1 term; a tilt must land the beam at +alpha r0 (Fresnel shift theorem),
  anisotropic waists on non-square grids pin x against y;
* ``two_heights``: two patches at different heights superpose their closed
  forms, each with its own r0 -- pins the per-point r0;
* ``separable``: column-only x jitter and row-only y jitter make the sum a
  product of two dense matrices;
* ``plane_identity``: u_I = exp(i k d1) equals folding exp(i k d1) into u1;
* ``single_point``: |u2| = |u1| / (lambda z0) everywhere;
* ``adjoint_dot_*``: <A u, g> = <u, A^H g> for random u, g, against the
  (independently pinned) forward -- true for the adjoint and no other map;
* ``window_*``: an off-axis destination window (centre x0, y0) -- a whole-pixel
  offset is the same sum at shifted pixel indices; a tilted Gaussian beam
  seen through a window centred near its landing point matches the closed form
  at the window's coordinates; the adjoint with a window passes the dot test;
* ``eq5_*``, ``eq2_*``: the sums that precede Eq. (7).  Eq. (5) keeps the exact
  output chirp, so a flat patch at height c gives exactly the Fresnel
  propagation over r0 = z0 - c times r0 / z0 (Gaussian closed form, per
  patch); the Huygens sum Eq. (2)-(3) tends to the same beam times z0 / r0 as
  the beam becomes paraxial, within the next terms of the expansion of r and
  1/r^2 (k rho^4 / (8 r0^3) and rho^2 / r0^2);
* ``line_*``: the one-dimensional forms -- the textbook 1D Gaussian beam (one
  axis factor of the 2D beam) with sqrt(r0 / z0) for Eq. (7) and (5) and
  z0 / r0 for the Huygens form, a tilt landing at +alpha r0, and a centred 1D
  DFT on a uniform line;
* ``adjoint_centred_dft``: on the centred-DFT geometry A = P F C with diagonal
  pre- and post-phases, so A^H g = conj(C) F^H (conj(P) g) with F^H the
  unnormalised inverse DFT (numpy.fft).

Every function takes an optional ``lib`` (an oracle variant) so that
``test_planted_mistakes`` can show each planted error fails some pin.
"""
import numpy as np

import oracle
import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# Textbook paraxial Gaussian beam, exp(+i k r) convention, written per axis so
# anisotropic waists factor: a 2D beam is exp(i k z) times the product of two
# 1D factors sqrt(w0/w) exp(-X^2/w^2) exp(i k X^2 / (2 R)) exp(-i zeta / 2),
# with w = w0 sqrt(1 + (z/zR)^2), 1/R = z / (z^2 + zR^2), zeta = atan(z/zR),
# zR = pi w0^2 / lambda.
# ---------------------------------------------------------------------------

def beam_1d(X, w0, lam, z):
    zr = np.pi * w0 * w0 / lam
    w = w0 * np.sqrt(1.0 + (z / zr) ** 2)
    inv_r = z / (z * z + zr * zr)
    zeta = np.arctan(z / zr)
    k = 2.0 * np.pi / lam
    return np.sqrt(w0 / w) * np.exp(-X * X / (w * w)) * np.exp(1j * (k * X * X * inv_r / 2.0 - zeta / 2.0))


def beam_2d(X, Y, w0x, w0y, lam, z, tilt=(0.0, 0.0)):
    """Propagation over z of exp(-x^2/w0x^2 - y^2/w0y^2) exp(i k (ax x + ay y)).

    A linear phase tilt shifts the beam to X - ax z and multiplies it by
    exp(i k (ax X - ax^2 z / 2)), per axis (Fresnel shift theorem).
    """
    k = 2.0 * np.pi / lam
    ax, ay = tilt
    tx = np.exp(1j * k * (ax * X - ax * ax * z / 2.0))
    ty = np.exp(1j * k * (ay * Y - ay * ay * z / 2.0))
    return (np.exp(1j * k * z) * beam_1d(X - ax * z, w0x, lam, z) * tx
            * beam_1d(Y - ay * z, w0y, lam, z) * ty)


def beam_line(X, w0, lam, z, tilt=0.0):
    """1D Fresnel propagation over z, exp(i k z) / sqrt(i lambda z) * integral, of
    exp(-x^2 / w0^2) exp(i k tilt x): one axis of ``beam_2d`` with its exp(i k z)."""
    k = 2.0 * np.pi / lam
    return (np.exp(1j * k * z) * beam_1d(X - tilt * z, w0, lam, z)
            * np.exp(1j * k * (tilt * X - tilt * tilt * z / 2.0)))


def flat_surface_factor(X, Y, z0, r0, lam):
    """F with (Eq. 7 sum for a flat source at height c, u_I = 1) * area = F * U(r0).

    For a flat source at height c (r0 = z0 - c) the Fourier-form sum is the
    Fresnel propagation U over r0 times r0 / z0 (amplitude 1/(lambda z0), not
    1/(lambda r0)) and times exp(i k |X|^2 (1/(2 z0) - 1/(2 r0))) (the output
    chirp of Eq. (6) instead of the exact one); exp(i k z0) exp(-i k c) is
    exp(i k r0).
    """
    k = 2.0 * np.pi / lam
    return (r0 / z0) * np.exp(1j * k * (X * X + Y * Y) * (1.0 / (2.0 * z0) - 1.0 / (2.0 * r0)))


def grid_axis(n, p, centre=0.0):
    return centre + p * (np.arange(n) - n / 2.0)


def gaussian_source(nx, ny, p1x, p1y, w0x, w0y, centre=(0.0, 0.0), tilt=(0.0, 0.0), lam=532e-9):
    k = 2.0 * np.pi / lam
    X, Y = np.meshgrid(grid_axis(nx, p1x, centre[0]), grid_axis(ny, p1y, centre[1]))
    u = np.exp(-((X - centre[0]) / w0x) ** 2 - ((Y - centre[1]) / w0y) ** 2)
    u = u * np.exp(1j * k * (tilt[0] * X + tilt[1] * Y))
    return X.reshape(-1), Y.reshape(-1), u.reshape(-1)


def dest_xy(mx, my, p2x, p2y):
    ix, iy = np.meshgrid(np.arange(mx), np.arange(my))
    return p2x * (ix.reshape(-1) - mx // 2), p2y * (iy.reshape(-1) - my // 2)


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def centred_dft(c, incident, lib=None):
    lam, z0 = 532e-9, 0.1
    nx, ny, p1x, p1y = 16, 12, 8e-6, 6e-6
    r0 = z0 - c
    p2x, p2y = lam * r0 / (nx * p1x), lam * r0 / (ny * p1y)
    X1, Y1 = np.meshgrid(p1x * (np.arange(nx) - nx // 2), p1y * (np.arange(ny) - ny // 2))
    rng = np.random.default_rng(3)
    u = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    got = oracle.direct_grid(X1.reshape(-1), Y1.reshape(-1), np.full(nx * ny, c), u.reshape(-1),
                             lam, z0, p2x, p2y, nx, ny, incident=incident, lib=lib)
    k = 2 * np.pi / lam
    g = u.astype(np.complex128) * np.exp(1j * k * (-c + (X1 ** 2 + Y1 ** 2) / (2 * r0)))
    if incident == "plane":
        g = g * np.exp(1j * k * c)
    S = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(g)))
    X, Y = dest_xy(nx, ny, p2x, p2y)
    post = np.exp(1j * k * (z0 + (X ** 2 + Y ** 2) / (2 * z0))) / (1j * lam * z0)
    return rel_l2(got, (post * S.reshape(-1)).reshape(ny, nx)), 1e-11


def gaussian_on_axis(lib=None):
    lam, z0, p1, w0, n = 532e-9, 0.1, 8e-6, 100e-6, 128
    x, y, u = gaussian_source(n, n, p1, p1, w0, w0, lam=lam)
    got = oracle.direct_grid(x, y, np.zeros_like(x), u, lam, z0, p1, p1, n, n,
                             incident="none", lib=lib) * p1 * p1
    X, Y = dest_xy(n, n, p1, p1)
    # k z0 ~ 1.2e6 rad is formed in FP64 on both sides: ~2e-10 rad of rounding
    return rel_l2(got, beam_2d(X, Y, w0, w0, lam, z0).reshape(n, n)), 1e-9


def gaussian_tilted_anisotropic(c, lib=None):
    lam, z0 = 532e-9, 0.1
    r0 = z0 - c
    tilt = (5e-4, -8e-4)
    x, y, u = gaussian_source(128, 160, 8e-6, 6.4e-6, 80e-6, 100e-6, tilt=tilt, lam=lam)
    mx, my, p2x, p2y = 100, 80, 10e-6, 12e-6
    got = oracle.direct_grid(x, y, np.full_like(x, c), u, lam, z0, p2x, p2y, mx, my,
                             incident="none", lib=lib) * 8e-6 * 6.4e-6
    X, Y = dest_xy(mx, my, p2x, p2y)
    want = flat_surface_factor(X, Y, z0, r0, lam) * beam_2d(X, Y, 80e-6, 100e-6, lam, r0, tilt)
    return rel_l2(got, want.reshape(my, mx)), 1e-9


def two_heights(lib=None):
    lam, z0, p1 = 633e-9, 0.25, 8e-6
    parts = [((-200e-6, 40e-6), 15e-6, 70e-6), ((180e-6, -60e-6), -40e-6, 90e-6)]
    xs, ys, ds, us = [], [], [], []
    for centre, c, w0 in parts:
        x, y, u = gaussian_source(112, 112, p1, p1, w0, w0, centre=centre, lam=lam)
        xs.append(x); ys.append(y); us.append(u); ds.append(np.full_like(x, c))
    x, y, d, u = map(np.concatenate, (xs, ys, ds, us))
    mx = my = 96
    p2 = 12e-6
    got = oracle.direct_grid(x, y, d, u, lam, z0, p2, p2, mx, my, incident="none", lib=lib) * p1 * p1
    X, Y = dest_xy(mx, my, p2, p2)
    want = np.zeros_like(X, dtype=np.complex128)
    for centre, c, w0 in parts:
        r0 = z0 - c
        # propagation is shift-invariant: a source centred at s gives U(X - s)
        want += flat_surface_factor(X, Y, z0, r0, lam) * beam_2d(
            X - centre[0], Y - centre[1], w0, w0, lam, r0)
    return rel_l2(got, want.reshape(my, mx)), 1e-9


def separable(lib=None):
    lam, z0 = 532e-9, 0.1
    nx, ny, mx, my = 20, 14, 18, 10
    rng = np.random.default_rng(11)
    xs = 8e-6 * (np.arange(nx) - (nx - 1) / 2) + rng.uniform(-2e-6, 2e-6, nx)
    ys = 7e-6 * (np.arange(ny) - (ny - 1) / 2) + rng.uniform(-2e-6, 2e-6, ny)
    X1, Y1 = np.meshgrid(xs, ys)
    u = synth.random_field(rng, nx, ny).reshape(ny, nx)
    p2x, p2y = 9e-6, 11e-6
    got = oracle.direct_grid(X1.reshape(-1), Y1.reshape(-1), np.zeros(nx * ny), u.reshape(-1),
                             lam, z0, p2x, p2y, mx, my, incident="none", lib=lib)
    k = 2 * np.pi / lam
    Xd = p2x * (np.arange(mx) - mx // 2)
    Yd = p2y * (np.arange(my) - my // 2)
    G = u.astype(np.complex128) * np.exp(1j * k * (X1 ** 2 + Y1 ** 2) / (2 * z0))
    Ax = np.exp(-1j * k * np.outer(Xd, xs) / z0)   # (mx, nx)
    Ay = np.exp(-1j * k * np.outer(Yd, ys) / z0)   # (my, ny)
    post = np.exp(1j * k * (z0 + (Xd[None, :] ** 2 + Yd[:, None] ** 2) / (2 * z0))) / (1j * lam * z0)
    return rel_l2(got, post * (Ay @ G @ Ax.T)), 1e-12


def plane_identity(lib=None):
    w = synth.config("sinusoid_128", side=24, out=16)
    k = 2 * np.pi / w.lam
    ix, iy = synth.sample_pixels(w.mx, w.my, 40)
    a = oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                      "plane", lib=lib)
    folded = w.u.astype(np.complex128) * np.exp(1j * k * w.d)
    b = oracle.direct(w.x, w.y, w.d, folded, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                      "none", lib=lib)
    # phases up to k (d + |x|^2 / 2 r0) ~ 1e3 rad, formed in two different ways
    return rel_l2(b, a), 1e-12


def single_point(lib=None):
    lam, z0 = 532e-9, 0.2
    x, y, d = np.array([37e-6]), np.array([-12e-6]), np.array([4e-6])
    u = np.array([0.6 - 0.3j], dtype=np.complex64)
    got = oracle.direct_grid(x, y, d, u, lam, z0, 8e-6, 8e-6, 16, 16, lib=lib)
    want = abs(complex(u[0])) / (lam * z0)
    return float(np.max(np.abs(np.abs(got) - want)) / want), 1e-12


def adjoint_dot(incident, lib=None):
    w = synth.config("sinusoid_128", side=10, out=8)
    rng = np.random.default_rng(11)
    errs = []
    ix, iy = np.meshgrid(np.arange(w.mx), np.arange(w.my))
    for _ in range(3):
        u = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
        g = rng.standard_normal((w.my, w.mx)) + 1j * rng.standard_normal((w.my, w.mx))
        au = oracle.direct(w.x, w.y, w.d, u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                           ix.reshape(-1), iy.reshape(-1), incident, lib=lib)
        ahg = oracle.adjoint(w.x, w.y, w.d, g, w.lam, w.z0, w.p2x, w.p2y, incident=incident, lib=lib)
        lhs = np.vdot(g.reshape(-1), au)
        rhs = np.vdot(ahg, u)
        errs.append(abs(lhs - rhs) / (np.linalg.norm(au) * np.linalg.norm(g)))
    # phases ~ k z0 ~ 1.2e6 rad are formed in two different groupings: ~1e-10 each
    return max(errs), 1e-9


def adjoint_centred_dft(incident, lib=None):
    lam, z0, c = 532e-9, 0.1, 15e-6
    nx, ny, p1x, p1y = 16, 12, 8e-6, 6e-6
    r0 = z0 - c
    p2x, p2y = lam * r0 / (nx * p1x), lam * r0 / (ny * p1y)
    X1, Y1 = np.meshgrid(p1x * (np.arange(nx) - nx // 2), p1y * (np.arange(ny) - ny // 2))
    rng = np.random.default_rng(5)
    g = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    got = oracle.adjoint(X1.reshape(-1), Y1.reshape(-1), np.full(nx * ny, c), g, lam, z0, p2x, p2y,
                         incident=incident, lib=lib).reshape(ny, nx)
    k = 2 * np.pi / lam
    pre = np.exp(1j * k * (-c + (X1 ** 2 + Y1 ** 2) / (2 * r0)))
    if incident == "plane":
        pre = pre * np.exp(1j * k * c)
    X, Y = dest_xy(nx, ny, p2x, p2y)
    post = (np.exp(1j * k * (z0 + (X ** 2 + Y ** 2) / (2 * z0))) / (1j * lam * z0)).reshape(ny, nx)
    h = np.conj(post) * g
    t = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(h))) * (nx * ny)
    # the oracle adds k z0 ~ 1.2e6 rad into each term's argument before sincos (FP64
    # ulp there ~ 2e-10 rad); the reference rounds it separately
    return rel_l2(got, np.conj(pre) * t), 5e-10


def window_integer_shift(lib=None):
    w = synth.config("sinusoid_128", side=20, out=16)
    a, b = 3, -2
    ix, iy = np.meshgrid(np.arange(w.mx), np.arange(w.my))
    ix, iy = ix.reshape(-1), iy.reshape(-1)
    got = oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                        lib=lib, x0=a * w.p2x, y0=b * w.p2y)
    want = oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix + a, iy + b,
                         lib=lib)
    # X formed as x0 + p2x (ix - m/2) or as p2x (ix + a - m/2): ulp-level phase differences
    return rel_l2(got, want), 1e-11


def window_offset_gaussian(lib=None):
    lam, z0, c = 532e-9, 0.1, 10e-6
    r0 = z0 - c
    tilt = (3e-3, -2e-3)                       # lands near (0.27 mm, -0.18 mm)
    x, y, u = gaussian_source(128, 160, 8e-6, 6.4e-6, 80e-6, 100e-6, tilt=tilt, lam=lam)
    mx, my, p2x, p2y = 100, 80, 10e-6, 12e-6
    x0, y0 = 0.2637e-3, -0.1743e-3            # not a whole number of pixels
    got = oracle.direct_grid(x, y, np.full_like(x, c), u, lam, z0, p2x, p2y, mx, my,
                             incident="none", lib=lib, x0=x0, y0=y0) * 8e-6 * 6.4e-6
    X, Y = dest_xy(mx, my, p2x, p2y)
    X, Y = X + x0, Y + y0
    want = flat_surface_factor(X, Y, z0, r0, lam) * beam_2d(X, Y, 80e-6, 100e-6, lam, r0, tilt)
    return rel_l2(got, want.reshape(my, mx)), 1e-9


def window_adjoint_dot(lib=None):
    w = synth.config("sinusoid_128", side=10, out=8)
    rng = np.random.default_rng(13)
    x0, y0 = 0.41e-3, -0.23e-3
    ix, iy = np.meshgrid(np.arange(w.mx), np.arange(w.my))
    u = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
    g = rng.standard_normal((w.my, w.mx)) + 1j * rng.standard_normal((w.my, w.mx))
    au = oracle.direct(w.x, w.y, w.d, u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                       ix.reshape(-1), iy.reshape(-1), lib=lib, x0=x0, y0=y0)
    ahg = oracle.adjoint(w.x, w.y, w.d, g, w.lam, w.z0, w.p2x, w.p2y, lib=lib, x0=x0, y0=y0)
    lhs, rhs = np.vdot(g.reshape(-1), au), np.vdot(ahg, u)
    return abs(lhs - rhs) / (np.linalg.norm(au) * np.linalg.norm(g)), 1e-9


def _patch(c, model, lib):
    """Tilted anisotropic Gaussian patch at height c through Eq. (5) or Eq. (2)."""
    lam, z0 = 532e-9, 0.1
    r0 = z0 - c
    tilt = (5e-4, -8e-4)
    x, y, u = gaussian_source(128, 160, 8e-6, 6.4e-6, 80e-6, 100e-6, tilt=tilt, lam=lam)
    mx, my, p2x, p2y = 100, 80, 10e-6, 12e-6
    got = oracle.surface(model, x, y, np.full_like(x, c), u, lam, z0, p2x, p2y, mx, my,
                         incident="none", lib=lib) * 8e-6 * 6.4e-6
    X, Y = dest_xy(mx, my, p2x, p2y)
    beam = beam_2d(X, Y, 80e-6, 100e-6, lam, r0, tilt).reshape(my, mx)
    return got, beam, r0, z0


def eq5_gaussian(c, lib=None):
    got, beam, r0, z0 = _patch(c, "eq5", lib)
    # exact up to the FP64 rounding of k z0 ~ 1.2e6 rad
    return rel_l2(got, (r0 / z0) * beam), 1e-9


def eq2_gaussian(c, lib=None):
    got, beam, r0, z0 = _patch(c, "eq2", lib)
    # Huygens vs its Fresnel limit: the beam (w ~ 230 um at r0) and the tilt keep
    # rho = |X - x| below ~0.5 mm where the field matters, so k rho^4 / (8 r0^3) + rho^2 / r0^2
    # is below ~1e-4 (5e-6 measured)
    return rel_l2(got, (z0 / r0) * beam), 1e-4


def eq_two_heights(model, lib=None):
    lam, z0, p1 = 633e-9, 0.25, 8e-6
    parts = [((-200e-6, 40e-6), 15e-6, 70e-6), ((180e-6, -60e-6), -40e-6, 90e-6)]
    xs, ys, ds, us = [], [], [], []
    for centre, c, w0 in parts:
        x, y, u = gaussian_source(112, 112, p1, p1, w0, w0, centre=centre, lam=lam)
        xs.append(x); ys.append(y); us.append(u); ds.append(np.full_like(x, c))
    x, y, d, u = map(np.concatenate, (xs, ys, ds, us))
    mx = my = 64
    p2 = 14e-6
    got = oracle.surface(model, x, y, d, u, lam, z0, p2, p2, mx, my, incident="none", lib=lib) * p1 * p1
    X, Y = dest_xy(mx, my, p2, p2)
    want = np.zeros_like(X, dtype=np.complex128)
    for centre, c, w0 in parts:
        r0 = z0 - c
        f = r0 / z0 if model == "eq5" else z0 / r0
        want += f * beam_2d(X - centre[0], Y - centre[1], w0, w0, lam, r0)
    return rel_l2(got, want.reshape(my, mx)), (1e-9 if model == "eq5" else 1e-4)


def surface_plane_identity(model, lib=None):
    w = synth.config("sinusoid_128", side=16, out=12)
    k = 2 * np.pi / w.lam
    a = oracle.surface(model, w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                       incident="plane", lib=lib)
    folded = w.u.astype(np.complex128) * np.exp(1j * k * w.d)
    b = oracle.surface(model, w.x, w.y, w.d, folded, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                       incident="none", lib=lib)
    # k r ~ 1.2e6 rad formed with and without k d added: ~1e-10
    return rel_l2(b, a), 1e-9


def line_gaussian(model, c, lib=None):
    lam, z0, p1, w0, tilt = 633e-9, 0.2, 10e-6, 120e-6, 6e-4
    r0 = z0 - c
    k = 2 * np.pi / lam
    x = grid_axis(256, p1)
    u = np.exp(-(x / w0) ** 2) * np.exp(1j * k * tilt * x)
    m, p2 = 200, 12e-6
    got = oracle.line(model, x, np.full_like(x, c), u, lam, z0, p2, m, incident="none", lib=lib) * p1
    X = p2 * (np.arange(m) - m // 2)
    beam = beam_line(X, w0, lam, r0, tilt)
    if model == "eq7":
        want = np.sqrt(r0 / z0) * np.exp(1j * k * X * X * (1 / (2 * z0) - 1 / (2 * r0))) * beam
    elif model == "eq5":
        want = np.sqrt(r0 / z0) * beam
    else:
        want = (z0 / r0) * beam
    # eq7/eq5: FP64 rounding of k z0 ~ 2e6 rad; eq2: its Fresnel limit, rho up to ~0.6 mm
    # where the field matters: k rho^4 / (8 r0^3) + rho^2 / r0^2 below ~1e-4
    return rel_l2(got, want), (1e-9 if model != "eq2" else 1e-4)


def line_centred_dft(c, lib=None):
    lam, z0, n, p1 = 633e-9, 0.2, 48, 10e-6
    r0 = z0 - c
    p2 = lam * r0 / (n * p1)
    x = p1 * (np.arange(n) - n // 2)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = oracle.line("eq7", x, np.full(n, c), u, lam, z0, p2, n, incident="plane", lib=lib)
    k = 2 * np.pi / lam
    g = u * np.exp(1j * k * x * x / (2 * r0))          # -k c and the incident k c cancel
    S = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(g)))
    X = p2 * (np.arange(n) - n // 2)
    post = np.exp(1j * k * (z0 + X * X / (2 * z0))) / np.sqrt(1j * lam * z0)
    # the oracle folds -pi/4 into the argument k (z0 + X^2 / (2 z0)) ~ 2e6 rad before sincos
    # (FP64 ulp there ~ 5e-10 rad); the reference divides by sqrt(i lambda z0) instead
    return rel_l2(got, post * S), 1e-9


def line_plane_identity(model, lib=None):
    rng = np.random.default_rng(8)
    x = np.sort(rng.uniform(-1e-3, 1e-3, 40))
    d = 30e-6 * np.sin(2 * np.pi * x / 0.7e-3)
    u = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    lam, z0, p2, m = 633e-9, 0.2, 10e-6, 24
    k = 2 * np.pi / lam
    a = oracle.line(model, x, d, u, lam, z0, p2, m, incident="plane", lib=lib)
    b = oracle.line(model, x, d, u * np.exp(1j * k * d), lam, z0, p2, m, incident="none", lib=lib)
    return rel_l2(b, a), 1e-9


PINS = {
    # cheap pins first: the planted-mistake test stops at the first pin that fails
    "centred_dft_flat_none": lambda lib=None: centred_dft(0.0, "none", lib),
    "centred_dft_raised_none": lambda lib=None: centred_dft(20e-6, "none", lib),
    "centred_dft_raised_plane": lambda lib=None: centred_dft(20e-6, "plane", lib),
    "separable": separable,
    "plane_identity": plane_identity,
    "single_point": single_point,
    "window_integer_shift": window_integer_shift,
    "window_adjoint_dot": window_adjoint_dot,
    "eq5_plane_identity": lambda lib=None: surface_plane_identity("eq5", lib),
    "eq2_plane_identity": lambda lib=None: surface_plane_identity("eq2", lib),
    "line_eq7_gaussian": lambda lib=None: line_gaussian("eq7", 25e-6, lib),
    "line_eq5_gaussian": lambda lib=None: line_gaussian("eq5", 25e-6, lib),
    "line_eq2_gaussian": lambda lib=None: line_gaussian("eq2", 25e-6, lib),
    "line_eq2_gaussian_flat": lambda lib=None: line_gaussian("eq2", 0.0, lib),
    "line_centred_dft": lambda lib=None: line_centred_dft(12e-6, lib),
    "line_eq7_plane_identity": lambda lib=None: line_plane_identity("eq7", lib),
    "line_eq5_plane_identity": lambda lib=None: line_plane_identity("eq5", lib),
    "line_eq2_plane_identity": lambda lib=None: line_plane_identity("eq2", lib),
    "adjoint_dot_plane": lambda lib=None: adjoint_dot("plane", lib),
    "adjoint_dot_none": lambda lib=None: adjoint_dot("none", lib),
    "adjoint_centred_dft_plane": lambda lib=None: adjoint_centred_dft("plane", lib),
    "adjoint_centred_dft_none": lambda lib=None: adjoint_centred_dft("none", lib),
    "gaussian_on_axis": gaussian_on_axis,
    "gaussian_tilted_raised": lambda lib=None: gaussian_tilted_anisotropic(20e-6, lib),
    "gaussian_tilted_lowered": lambda lib=None: gaussian_tilted_anisotropic(-35e-6, lib),
    "two_heights": two_heights,
    "window_offset_gaussian": window_offset_gaussian,
    "eq5_gaussian_raised": lambda lib=None: eq5_gaussian(20e-6, lib),
    "eq5_gaussian_lowered": lambda lib=None: eq5_gaussian(-35e-6, lib),
    "eq2_gaussian_raised": lambda lib=None: eq2_gaussian(20e-6, lib),
    "eq2_gaussian_lowered": lambda lib=None: eq2_gaussian(-35e-6, lib),
    "eq5_two_heights": lambda lib=None: eq_two_heights("eq5", lib),
    "eq2_two_heights": lambda lib=None: eq_two_heights("eq2", lib),
}
