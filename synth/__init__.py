"""Seeded synthetic source surfaces for the arbitrary-shape-surface Fresnel sum.

This module only draws inputs: sample positions (x1, y1), the surface
displacement d1(x1, y1) and the complex source field u1, plus the optical
parameters they come with.  It holds none of the diffraction arithmetic, so
both the CPU oracle's tests and the GPU path's tests and benchmark can use it
without sharing any of the method's code.

Conventions (shared by every generator here):
  * a source grid has ``nx`` columns and ``ny`` rows; arrays are flattened in
    row-major (iy, ix) order with ix fastest;
  * nominal positions are symmetric about the optical axis,
    ``x = pitch * (ix - (nx - 1) / 2)`` (and likewise for y), plus a uniform
    jitter drawn per point and per axis;
  * the random draws happen in a fixed order -- jitter_x, jitter_y, amplitude
    (or mask), phase -- each of shape (ny, nx), from
    ``numpy.random.default_rng(seed)`` (PCG64);
  * d1 is evaluated at the jittered position;
  * u1 is cast to complex64 once; every consumer uses that same array.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "jittered_grid",
    "sinusoidal_relief",
    "spherical_cap",
    "random_field",
    "config",
    "CONFIG_NAMES",
    "sample_pixels",
    "LineWorkload",
    "facet_profile",
    "quadratic_profile",
    "line_config",
    "LINE_CONFIG_NAMES",
    "zernike_height",
    "zernike_basis",
    "smooth_phase",
    "warm_pair_geometry",
]


@dataclass
class Workload:
    """One synthetic problem: source samples, optics and destination grid."""

    name: str
    x: np.ndarray          # float64 [n]  source x1 (m)
    y: np.ndarray          # float64 [n]  source y1 (m)
    d: np.ndarray          # float64 [n]  surface displacement d1(x1) (m)
    u: np.ndarray          # complex64 [n] source field u1
    lam: float             # wavelength (m)
    z0: float              # source-to-destination distance (m)
    p2x: float             # destination pitch along x (m)
    p2y: float             # destination pitch along y (m)
    mx: int                # destination columns
    my: int                # destination rows
    tol: float = 1e-5      # requested accuracy (relative L2)
    incident: str = "plane"  # "plane": u_I = exp(i k d1); "none": u_I = 1
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def jittered_grid(rng: np.random.Generator, nx: int, ny: int, pitch: float,
                  jitter: float, pitch_y: float | None = None):
    """Positions of an nx-by-ny grid with uniform jitter in [-jitter, jitter).

    Draws jitter_x then jitter_y, each of shape (ny, nx).  Returns flattened
    float64 arrays (x, y) in row-major order.
    """
    py = pitch if pitch_y is None else pitch_y
    jx = rng.uniform(-jitter, jitter, size=(ny, nx)) if jitter > 0 else np.zeros((ny, nx))
    jy = rng.uniform(-jitter, jitter, size=(ny, nx)) if jitter > 0 else np.zeros((ny, nx))
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    x = pitch * (ix[None, :] - (nx - 1) / 2.0) + jx
    y = py * (iy[:, None] - (ny - 1) / 2.0) + jy
    return x.reshape(-1).astype(np.float64), y.reshape(-1).astype(np.float64)


def sinusoidal_relief(x: np.ndarray, y: np.ndarray, amplitude: float, period: float) -> np.ndarray:
    """d1 = A sin(2 pi x / period) cos(2 pi y / period)."""
    return amplitude * np.sin(2.0 * np.pi * x / period) * np.cos(2.0 * np.pi * y / period)


def spherical_cap(x: np.ndarray, y: np.ndarray, radius: float) -> np.ndarray:
    """d1 = R - sqrt(R^2 - x^2 - y^2): sag of a sphere of radius R (R > |x|)."""
    return radius - np.sqrt(radius * radius - x * x - y * y)


def random_field(rng: np.random.Generator, nx: int, ny: int, amplitude: str = "uniform") -> np.ndarray:
    """Complex64 source field: amplitude then phase U[0, 2 pi), each (ny, nx).

    amplitude = "uniform" draws U[0, 1); "binary" draws a Bernoulli(0.5) mask in {0, 1}.
    """
    if amplitude == "uniform":
        amp = rng.uniform(0.0, 1.0, size=(ny, nx))
    elif amplitude == "binary":
        amp = (rng.uniform(0.0, 1.0, size=(ny, nx)) < 0.5).astype(np.float64)
    else:
        raise ValueError(f"unknown amplitude kind {amplitude!r}")
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    u = amp * np.exp(1j * phase)
    return u.reshape(-1).astype(np.complex64)


# ---------------------------------------------------------------------------
# The three benchmark surfaces.  Each takes a ``side`` override so tests can run
# the same geometry family at a size the CPU oracle finishes quickly; the
# destination grid follows the source side unless given.
# ---------------------------------------------------------------------------

def _sinusoid_128(seed: int = 0, side: int = 128, out: int | None = None) -> Workload:
    """128^2 sinusoidal relief: 8 um pitch, +-2.4 um jitter, A = 50 um, period 1 mm,
    uniform amplitude and phase, lambda = 532 nm, z0 = 0.1 m, 8 um destination pitch."""
    rng = np.random.default_rng(seed)
    p = 8e-6
    x, y = jittered_grid(rng, side, side, p, 2.4e-6)
    d = sinusoidal_relief(x, y, 50e-6, 1e-3)
    u = random_field(rng, side, side, "uniform")
    m = side if out is None else out
    return Workload("sinusoid_128", x, y, d, u, 532e-9, 0.1, p, p, m, m, 1e-5, "plane",
                    {"side": side, "seed": seed})


def _cap_2048(seed: int = 0, side: int = 2048, out: int | None = None) -> Workload:
    """2048^2 spherical cap R = 50 mm: 8 um pitch, +-0.3 pitch jitter, binary amplitude
    mask with uniform phase, lambda = 532 nm, z0 = 0.2 m, 8 um destination pitch."""
    rng = np.random.default_rng(seed)
    p = 8e-6
    x, y = jittered_grid(rng, side, side, p, 0.3 * p)
    d = spherical_cap(x, y, 50e-3)
    u = random_field(rng, side, side, "binary")
    m = side if out is None else out
    return Workload("cap_2048", x, y, d, u, 532e-9, 0.2, p, p, m, m, 1e-5, "plane",
                    {"side": side, "seed": seed})


def _sinusoid_4096(seed: int = 0, side: int = 4096, out: int | None = None) -> Workload:
    """4096^2 sinusoidal relief: 4 um pitch, +-0.3 pitch jitter, A = 30 um, period 0.5 mm,
    uniform amplitude and phase, lambda = 633 nm, z0 = 0.3 m, 4 um destination pitch."""
    rng = np.random.default_rng(seed)
    p = 4e-6
    x, y = jittered_grid(rng, side, side, p, 0.3 * p)
    d = sinusoidal_relief(x, y, 30e-6, 0.5e-3)
    u = random_field(rng, side, side, "uniform")
    m = side if out is None else out
    return Workload("sinusoid_4096", x, y, d, u, 633e-9, 0.3, p, p, m, m, 1e-5, "plane",
                    {"side": side, "seed": seed})


def smooth_target(rng: np.random.Generator, nx: int, ny: int, sigma_px: float = 4.0) -> np.ndarray:
    """Target intensity (ny, nx) float64 in [0, 1]: uniform noise U[0, 1) filtered by a
    periodic Gaussian of standard deviation sigma_px pixels, rescaled to [0, 1]."""
    noise = rng.uniform(0.0, 1.0, size=(ny, nx))
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.fftfreq(nx)[None, :]
    gain = np.exp(-2.0 * (np.pi * sigma_px) ** 2 * (fx * fx + fy * fy))
    t = np.real(np.fft.ifft2(np.fft.fft2(noise) * gain))
    t -= t.min()
    return t / t.max()


def _holo_1024(seed: int = 0, side: int = 1024, out: int | None = None) -> Workload:
    """Phase-hologram problem: 1024^2 phase-only source on a spherical cap R = 80 mm,
    8 um pitch with +-0.3 pitch jitter, unit amplitude, zero initial phase,
    lambda = 532 nm, z0 = 0.15 m, 1024^2 destination at 8 um; the target intensity
    (Gaussian-filtered uniform noise, sigma 4 px) is in meta["target"]."""
    rng = np.random.default_rng(seed)
    p = 8e-6
    x, y = jittered_grid(rng, side, side, p, 0.3 * p)
    d = spherical_cap(x, y, 80e-3)
    u = np.ones(side * side, dtype=np.complex64)
    m = side if out is None else out
    target = smooth_target(rng, m, m, 4.0)
    return Workload("holo_1024", x, y, d, u, 532e-9, 0.15, p, p, m, m, 1e-5, "plane",
                    {"side": side, "seed": seed, "target": target})


_CONFIGS = {
    "sinusoid_128": _sinusoid_128,
    "cap_2048": _cap_2048,
    "sinusoid_4096": _sinusoid_4096,
    "holo_1024": _holo_1024,
}
CONFIG_NAMES = tuple(_CONFIGS)


def config(name: str, seed: int = 0, side: int | None = None, out: int | None = None) -> Workload:
    """Build a named benchmark surface (optionally at a reduced side length)."""
    fn = _CONFIGS[name]
    kw = {"seed": seed, "out": out}
    if side is not None:
        kw["side"] = side
    return fn(**kw)


def sample_pixels(mx: int, my: int, count: int, seed: int = 1):
    """Distinct random destination pixels (ix, iy) as int32 arrays, sorted by flat index."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(mx * my, size=min(count, mx * my), replace=False)
    flat.sort()
    return (flat % mx).astype(np.int32), (flat // mx).astype(np.int32)


# ---------------------------------------------------------------------------
# One-dimensional profiles (a line source x1 with displacement d1(x1)), sampled
# uniformly along the surface: equal arc length p between neighbours, so the
# spacing in x1 shrinks to p |cos theta| where the surface is tilted by theta.
# ---------------------------------------------------------------------------

@dataclass
class LineWorkload:
    """One 1D problem: source samples along a profile, optics and destination line."""

    name: str
    x: np.ndarray          # float64 [n] source x1 (m)
    d: np.ndarray          # float64 [n] displacement d1(x1) (m)
    u: np.ndarray          # complex64 [n] source field u1
    lam: float
    z0: float
    p2: float              # destination pitch (m)
    m: int                 # destination pixels
    tol: float = 1e-5
    incident: str = "plane"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def facet_profile(angles_deg, points_per_facet: int, pitch: float):
    """Consecutive planar facets tilted by ``angles_deg`` to the x1 axis, each with
    ``points_per_facet`` samples at arc-length pitch ``pitch`` (samples at the
    middle of each arc step, so joints fall between samples).  The profile is
    continuous; it is shifted so that x1 and d1 both have mean zero.
    Returns (x, d) float64 arrays in order along the profile."""
    xs, ds = [], []
    x_start = d_start = 0.0
    for a in np.deg2rad(np.asarray(angles_deg, dtype=np.float64)):
        t = pitch * (np.arange(points_per_facet) + 0.5)
        xs.append(x_start + t * np.cos(a))
        ds.append(d_start + t * np.sin(a))
        x_start += points_per_facet * pitch * np.cos(a)
        d_start += points_per_facet * pitch * np.sin(a)
    x, d = np.concatenate(xs), np.concatenate(ds)
    return x - x.mean(), d - d.mean()


def _parabola_arc(x, a):
    """Arc length of d = a x^2 from the vertex to x (signed)."""
    t = 2.0 * a * x
    return (x * np.sqrt(1.0 + t * t)) / 2.0 + np.arcsinh(t) / (4.0 * a)


def quadratic_profile(n: int, pitch: float, a: float, newton_steps: int = 60):
    """d1 = a x1^2 sampled at arc lengths pitch (i - (n-1)/2) from the vertex,
    the x1 found by Newton's method on the closed-form arc length (ds/dx =
    sqrt(1 + (2 a x)^2)).  Returns (x, d) float64."""
    s_target = pitch * (np.arange(n) - (n - 1) / 2.0)
    x = s_target.copy()
    for _ in range(newton_steps):
        x = x - (_parabola_arc(x, a) - s_target) / np.sqrt(1.0 + (2.0 * a * x) ** 2)
    return x, a * x * x


def _facets_1d(seed: int = 0, points: int = 128) -> LineWorkload:
    """Four planar facets of 128 points tilted -30, -50, 0 and +50 degrees, 10 um
    arc pitch, unit field, lambda = 633 nm, z0 = 1 m, 1024 destination pixels at 10 um."""
    x, d = facet_profile((-30.0, -50.0, 0.0, 50.0), points, 10e-6)
    u = np.ones(x.shape[0], dtype=np.complex64)
    return LineWorkload("facets_1d", x, d, u, 633e-9, 1.0, 10e-6, 1024, 1e-5, "plane",
                        {"points_per_facet": points})


def _quadratic_1d(seed: int = 0, n: int = 1024, a: float = 100.0) -> LineWorkload:
    """d1 = a x1^2 (a = 100 / m, slope about +-0.9 at the ends), 1024 points at
    10 um arc pitch, unit field, lambda = 633 nm, z0 = 1 m, 1024 pixels at 10 um."""
    x, d = quadratic_profile(n, 10e-6, a)
    u = np.ones(n, dtype=np.complex64)
    return LineWorkload("quadratic_1d", x, d, u, 633e-9, 1.0, 10e-6, 1024, 1e-5, "plane",
                        {"a": a})


_LINE_CONFIGS = {"facets_1d": _facets_1d, "quadratic_1d": _quadratic_1d}
LINE_CONFIG_NAMES = tuple(_LINE_CONFIGS)


def line_config(name: str, **kw) -> LineWorkload:
    """Build a named 1D profile (keyword overrides go to its generator)."""
    return _LINE_CONFIGS[name](**kw)


# ---------------------------------------------------------------------------
# Inputs of the learned warm start: random surfaces (Zernike height maps) and
# random smooth source phases whose intensities the forward method produces.
# ---------------------------------------------------------------------------

def _zernike_radial(n: int, m: int, rho: np.ndarray) -> np.ndarray:
    from math import factorial
    out = np.zeros_like(rho)
    for k in range((n - m) // 2 + 1):
        c = (-1) ** k * factorial(n - k) / (factorial(k) * factorial((n + m) // 2 - k) * factorial((n - m) // 2 - k))
        out += c * rho ** (n - 2 * k)
    return out


def zernike_basis(x: np.ndarray, y: np.ndarray, radius: float, max_order: int = 6) -> np.ndarray:
    """The Zernike polynomials of radial orders 1 .. max_order (piston excluded) on the disc
    of the given radius (continued outside it) at the points (x, y): array (terms, n)."""
    rho = np.hypot(x, y) / radius
    th = np.arctan2(y, x)
    rows = []
    for n in range(1, max_order + 1):
        for m in range(-n, n + 1, 2):
            r = _zernike_radial(n, abs(m), rho)
            rows.append(r * (np.cos(m * th) if m >= 0 else np.sin(-m * th)))
    return np.array(rows)


def zernike_height(rng: np.random.Generator, x: np.ndarray, y: np.ndarray, radius: float,
                   max_order: int = 6, max_abs: float = 60e-6, basis: np.ndarray | None = None) -> np.ndarray:
    """Height map d1(x, y): a sum of the Zernike polynomials of radial order <= max_order
    (piston excluded) with standard-normal coefficients, scaled so that
    max |d1| = max_abs * U(0.2, 1).  `basis` (from zernike_basis on the same points)
    saves re-evaluating the polynomials."""
    z = zernike_basis(x, y, radius, max_order) if basis is None else basis
    d = rng.standard_normal(z.shape[0]) @ z
    scale = max_abs * rng.uniform(0.2, 1.0) / max(np.abs(d).max(), 1e-30)
    return d * scale


def smooth_phase(rng: np.random.Generator, nx: int, ny: int, sigma_px: float = 6.0,
                 amplitude: float = 3.0) -> np.ndarray:
    """Phase (ny, nx) float64: standard-normal noise filtered by a periodic Gaussian of
    sigma_px pixels, scaled to standard deviation `amplitude` radians."""
    noise = rng.standard_normal((ny, nx))
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.fftfreq(nx)[None, :]
    gain = np.exp(-2.0 * (np.pi * sigma_px) ** 2 * (fx * fx + fy * fy))
    ph = np.real(np.fft.ifft2(np.fft.fft2(noise) * gain))
    return ph * (amplitude / max(ph.std(), 1e-30))


def warm_pair_geometry(side: int = 512, seed: int = 0):
    """Source grid of the warm-start problems: side^2 samples at 8 um with +-0.3 pitch
    jitter, lambda = 532 nm, z0 = 0.1 m, side^2 destination at 8 um.  Returns
    (x, y, lam, z0, p2, m); heights come from zernike_height on this grid."""
    rng = np.random.default_rng(seed)
    p = 8e-6
    x, y = jittered_grid(rng, side, side, p, 0.3 * p)
    return x, y, 532e-9, 0.1, p, side
