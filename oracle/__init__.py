"""CPU oracle for the arbitrary-shape-surface Fresnel sum -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package.  The GPU path shares no code with it.

``direct`` evaluates Eq. (7) of Shimobaba, Masuda and Ito (Sec. 2) -- the
Fourier-form Fresnel sum from an arbitrary source surface, with the Fresnel
expansion of Eq. (4), r^2 ~ z0^2 in the amplitude, the output chirp of Eq. (6)
and the normal plane-wave incidence u_I = exp(i k d1) -- as the plain FP64 direct
sum over source points, one sincos per term, at any set of destination pixels.
It is written in C (``asf_oracle.c``) and parallel over pixels with OpenMP.

``adjoint`` evaluates the adjoint of that linear map, g1 = A^H g2, the same
way (one sincos per term, parallel over source points): the backward of the
forward with respect to u1.

``surface`` evaluates the two direct sums that precede Eq. (7): Eq. (5)
(Fresnel on the surface, before the output-chirp approximation) and Eq. (2)-(3)
(the Huygens sum on the surface, no expansion of r).  ``line`` evaluates the
one-dimensional forms of Eq. (7), (5) and (2) used by the paper's profiles
(Sec. 3), read as a surface that does not vary along y (the y integral done
analytically; see ``asf_oracle.c``).  These serve the approximation study.

``mp_direct`` is the same definition at 50 significant digits with mpmath, for
tiny inputs only: it checks the FP64 rounding of ``direct``, not its formula.
The formula itself is pinned by the tests in ``tests/test_oracle_pins.py``
(centred DFT, textbook Gaussian-beam propagation, shift theorem, separable
matrix form, invariants).

Readings of the paper taken here: the x1.x2 term carries a minus sign (Eq. (4),
(5), (9); Eq. (7) prints a plus); unit quadrature weights; destination pixel
(ix, iy) at X = x0 + p2x (ix - mx // 2), Y = y0 + p2y (iy - my // 2), with the
window centre (x0, y0) = 0 unless given.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asf_oracle.c")
_LIB = os.path.join(_HERE, "_asf_oracle.so")
_lib = None

INCIDENT = {"plane": 0, "none": 1}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math) into ``_asf_oracle.so``."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def load_library(path: str):
    """Open a compiled oracle library (the built one, or a test's own variant)."""
    lib = ctypes.CDLL(path)
    lib.asf_oracle_direct.restype = ctypes.c_int
    lib.asf_oracle_direct.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_double, ctypes.c_double,
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.asf_oracle_adjoint.restype = ctypes.c_int
    lib.asf_oracle_adjoint.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.asf_oracle_surface.restype = ctypes.c_int
    lib.asf_oracle_surface.argtypes = [ctypes.c_int32] + lib.asf_oracle_direct.argtypes
    lib.asf_oracle_line.restype = ctypes.c_int
    lib.asf_oracle_line.argtypes = [
        ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
        ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.asf_oracle_threads.restype = ctypes.c_int
    lib.asf_oracle_threads.argtypes = [ctypes.c_int32]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load_library(_LIB)
    return _lib


def threads(requested: int = 0) -> int:
    """Threads the oracle uses for ``requested`` (0 = OpenMP default)."""
    return int(_load().asf_oracle_threads(int(requested)))


def direct(x, y, d, u, lam, z0, p2x, p2y, mx, my, ix, iy, incident="plane", nthreads=0,
           lib=None, x0=0.0, y0=0.0):
    """u2 at destination pixels (ix[e], iy[e]) by the direct FP64 sum of Eq. (7).

    x, y, d: float64 [n] source coordinates and displacement (m); u: complex [n]
    source field (complex64 input is promoted exactly to complex128); ix, iy: int [n_eval];
    (x0, y0): the destination window's centre, pixel (ix, iy) at x0 + p2x (ix - mx // 2), ...
    Returns complex128 [n_eval].  Raises ValueError if some z0 - d <= 0.
    ``lib`` selects another compiled variant (tests only); default: the built oracle.
    """
    lib = _load() if lib is None else lib
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    ix = np.ascontiguousarray(ix, dtype=np.int32).reshape(-1)
    iy = np.ascontiguousarray(iy, dtype=np.int32).reshape(-1)
    n = x.shape[0]
    if not (y.shape[0] == n and d.shape[0] == n and u.shape[0] == n):
        raise ValueError("x, y, d, u must have equal length")
    if ix.shape != iy.shape:
        raise ValueError("ix and iy must have equal length")
    out = np.empty(2 * ix.shape[0], dtype=np.float64)
    rc = lib.asf_oracle_direct(
        n, x.ctypes.data, y.ctypes.data, d.ctypes.data, u.ctypes.data,
        float(lam), float(z0), float(p2x), float(p2y), float(x0), float(y0), int(mx), int(my),
        INCIDENT[incident], ix.shape[0], ix.ctypes.data, iy.ctypes.data,
        out.ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid arguments or r0 = z0 - d1 <= 0")
    return out.view(np.complex128)


SURFACE_MODELS = {"eq5": 5, "eq2": 2}
LINE_MODELS = {"eq7": 7, "eq5": 5, "eq2": 2}


def surface(model, x, y, d, u, lam, z0, p2x, p2y, mx, my, ix=None, iy=None, incident="plane",
            nthreads=0, lib=None, x0=0.0, y0=0.0):
    """u2 by Eq. (5) (``model="eq5"``) or the Huygens sum Eq. (2)-(3) (``"eq2"``).

    Arguments as for ``direct``; ix, iy default to the whole grid, in which case
    the result has shape (my, mx), else (n_eval,).
    """
    lib = _load() if lib is None else lib
    whole = ix is None
    if whole:
        gx, gy = np.meshgrid(np.arange(mx), np.arange(my))
        ix, iy = gx.reshape(-1), gy.reshape(-1)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    ix = np.ascontiguousarray(ix, dtype=np.int32).reshape(-1)
    iy = np.ascontiguousarray(iy, dtype=np.int32).reshape(-1)
    n = x.shape[0]
    if not (y.shape[0] == n and d.shape[0] == n and u.shape[0] == n) or ix.shape != iy.shape:
        raise ValueError("x, y, d, u (and ix, iy) must have equal length")
    out = np.empty(2 * ix.shape[0], dtype=np.float64)
    rc = lib.asf_oracle_surface(
        SURFACE_MODELS[model], n, x.ctypes.data, y.ctypes.data, d.ctypes.data, u.ctypes.data,
        float(lam), float(z0), float(p2x), float(p2y), float(x0), float(y0), int(mx), int(my),
        INCIDENT[incident], ix.shape[0], ix.ctypes.data, iy.ctypes.data, out.ctypes.data,
        int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid arguments or r0 = z0 - d1 <= 0")
    vals = out.view(np.complex128)
    return vals.reshape(my, mx) if whole else vals


def line(model, x, d, u, lam, z0, p2, m, ix=None, incident="plane", nthreads=0, lib=None, x0=0.0):
    """One-dimensional u2 at pixels ix (default: all m) by Eq. (7), (5) or (2) read in 1D.

    Eq. (7) and (5) in 1D are the exact (Fresnel chirp) integrals over y of the 2D forms,
    with the amplitude's r0 read as z0 as the 2D forms read it; Eq. (2) in 1D is
    an approximation the oracle makes itself: the y-integral of exp(i k R) / R^2 is
    taken by its stationary-phase leading term, relative error about 1 / (k rho)
    (1e-7 at rho = 1 m for visible light), far below the errors the study compares.
    x, d: float64 [n] (m); u: complex [n]; pixel ix at X = x0 + p2 (ix - m // 2).
    Returns complex128 [len(ix)].
    """
    lib = _load() if lib is None else lib
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    ix = np.arange(m, dtype=np.int32) if ix is None else np.ascontiguousarray(ix, dtype=np.int32).reshape(-1)
    n = x.shape[0]
    if not (d.shape[0] == n and u.shape[0] == n):
        raise ValueError("x, d, u must have equal length")
    out = np.empty(2 * ix.shape[0], dtype=np.float64)
    rc = lib.asf_oracle_line(
        LINE_MODELS[model], n, x.ctypes.data, d.ctypes.data, u.ctypes.data, float(lam), float(z0),
        float(p2), float(x0), int(m), INCIDENT[incident], ix.shape[0], ix.ctypes.data,
        out.ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid arguments or r0 = z0 - d1 <= 0")
    return out.view(np.complex128)


def direct_grid(x, y, d, u, lam, z0, p2x, p2y, mx, my, ix_range=None, iy_range=None,
                incident="plane", nthreads=0, lib=None, x0=0.0, y0=0.0):
    """u2 on the rectangle ix_range x iy_range (default: the whole grid), shape (rows, cols)."""
    ixs = np.arange(mx) if ix_range is None else np.asarray(list(ix_range))
    iys = np.arange(my) if iy_range is None else np.asarray(list(iy_range))
    gx, gy = np.meshgrid(ixs, iys)
    vals = direct(x, y, d, u, lam, z0, p2x, p2y, mx, my, gx.reshape(-1), gy.reshape(-1),
                  incident, nthreads, lib, x0, y0)
    return vals.reshape(len(iys), len(ixs))


def crop_gemm(x, y, d, u, lam, z0, p2x, p2y, mx, my, ix_range, iy_range, incident="plane",
              x0=0.0, y0=0.0, nthreads=0, chunk=8192):
    """u2 on the rectangle ix_range x iy_range by Eq. (7) written as FP64 matrix products.

    The same sum as ``direct``.  The cross term of the phase is separable,
    exp(-i k (x X + y Y) / r0) = exp(-i k x X / r0) exp(-i k y Y / r0), so over a
    rectangle of pixels
        S[Y, X] = sum_j Ay[j, Y] c_j Ax[j, X],   c_j = u_j u_I,j exp(i k (-d_j + |x_j|^2 / (2 r0_j)))
    is one complex matrix product Ay^T diag(c) Ax per chunk of source points
    (``numpy.matmul``), with every factor an explicit FP64 ``exp`` of its own
    argument.  The chunks' partial sums are added in point order.  The result is
    then multiplied by the post-phase exp(i k (z0 + (X^2 + Y^2) / (2 z0))) / (i lambda z0).
    Returns complex128 (rows, cols).  Raises ValueError if some z0 - d <= 0.
    """
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits

    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    n = x.shape[0]
    if not (y.shape[0] == n and d.shape[0] == n and u.shape[0] == n):
        raise ValueError("x, y, d, u must have equal length")
    if not np.all(z0 - d > 0.0):
        raise ValueError("oracle: r0 = z0 - d1 <= 0")
    k = 2.0 * np.pi / lam
    ixs = np.asarray(list(ix_range), dtype=np.int64)
    iys = np.asarray(list(iy_range), dtype=np.int64)
    X = x0 + p2x * (ixs - mx // 2).astype(np.float64)
    Y = y0 + p2y * (iys - my // 2).astype(np.float64)
    starts = list(range(0, n, chunk))

    def part(j0):
        sl = slice(j0, min(j0 + chunk, n))
        xj, yj, dj = x[sl], y[sl], d[sl]
        r0 = z0 - dj
        arg = k * (-dj + (xj * xj + yj * yj) / (2.0 * r0))
        if incident == "plane":
            arg = arg + k * dj
        c = u[sl] * np.exp(1j * arg)
        ax = np.exp(-1j * k * (np.outer(xj, X) / r0[:, None]))      # (chunk, cols)
        ay = np.exp(-1j * k * (np.outer(yj, Y) / r0[:, None]))      # (chunk, rows)
        return (ay * c[:, None]).T @ ax                               # (rows, cols)

    workers = threads(nthreads)
    with threadpool_limits(limits=1, user_api="blas"):
        with ThreadPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(part, starts))
    S = np.zeros((len(iys), len(ixs)), dtype=np.complex128)
    for p in parts:
        S += p
    post = np.exp(1j * k * (z0 + (X[None, :] ** 2 + Y[:, None] ** 2) / (2.0 * z0))) / (1j * lam * z0)
    return post * S


def adjoint(x, y, d, g2, lam, z0, p2x, p2y, jidx=None, incident="plane", nthreads=0, lib=None,
            x0=0.0, y0=0.0):
    """g1 = A^H g2 at source points jidx (default: all), by the direct FP64 sum.

    A is the linear map u1 -> u2 that ``direct`` evaluates; g2: complex [my, mx]
    (row-major, complex64 promoted exactly).  Returns complex128 [len(jidx)].
    """
    lib = _load() if lib is None else lib
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    g2 = np.ascontiguousarray(g2, dtype=np.complex128)
    if g2.ndim != 2:
        raise ValueError("g2 must be [my, mx]")
    my, mx = g2.shape
    n = x.shape[0]
    if not (y.shape[0] == n and d.shape[0] == n):
        raise ValueError("x, y, d must have equal length")
    jidx = np.arange(n, dtype=np.int64) if jidx is None else np.ascontiguousarray(jidx, dtype=np.int64).reshape(-1)
    out = np.empty(2 * jidx.shape[0], dtype=np.float64)
    rc = lib.asf_oracle_adjoint(
        n, x.ctypes.data, y.ctypes.data, d.ctypes.data, float(lam), float(z0), float(p2x),
        float(p2y), float(x0), float(y0), int(mx), int(my), INCIDENT[incident], g2.ctypes.data, jidx.shape[0],
        jidx.ctypes.data, out.ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid arguments or r0 = z0 - d1 <= 0")
    return out.view(np.complex128)


def mp_direct(x, y, d, u, lam, z0, p2x, p2y, mx, my, ix, iy, incident="plane", dps=50):
    """The same sum as ``direct`` in mpmath at ``dps`` digits (tiny inputs only).

    The FP64 inputs are taken as exact binary values (u as complex128).
    """
    import mpmath as mp

    with mp.workdps(dps):
        k = 2 * mp.pi / mp.mpf(lam)
        z0m = mp.mpf(z0)
        lamm = mp.mpf(lam)
        out = []
        for e in range(len(ix)):
            X = mp.mpf(p2x) * (int(ix[e]) - int(mx) // 2)
            Y = mp.mpf(p2y) * (int(iy[e]) - int(my) // 2)
            s = mp.mpc(0)
            for j in range(len(x)):
                xj, yj, dj = mp.mpf(float(x[j])), mp.mpf(float(y[j])), mp.mpf(float(d[j]))
                r0 = z0m - dj
                arg = k * (-dj + (xj * xj + yj * yj) / (2 * r0) - (xj * X + yj * Y) / r0)
                if incident == "plane":
                    arg += k * dj
                uj = complex(np.complex128(u[j]))
                s += mp.mpc(uj.real, uj.imag) * mp.expj(arg)
            post = mp.expj(k * (z0m + (X * X + Y * Y) / (2 * z0m))) / (mp.mpc(0, 1) * lamm * z0m)
            out.append(complex(post * s))
        return np.array(out, dtype=np.complex128)
