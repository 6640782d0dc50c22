"""CPU checks of the one-dimensional profile generators: samples are equally
spaced along the surface (arc length), which makes their x1 spacing shrink to
p |cos theta| on a facet tilted by theta (Sec. 2-3)."""
import numpy as np

import synth


def test_facets_arc_pitch_and_tilt():
    angles = (-30.0, -50.0, 0.0, 50.0)
    x, d = synth.facet_profile(angles, 128, 10e-6)
    assert x.shape == (512,) and np.all(np.diff(x) > 0)
    assert abs(x.mean()) < 1e-15 and abs(d.mean()) < 1e-15
    for f, a in enumerate(np.deg2rad(angles)):
        xs, ds = x[128 * f:128 * (f + 1)], d[128 * f:128 * (f + 1)]
        # within a facet: step p along the surface, p cos(theta) in x1, slope tan(theta)
        assert np.allclose(np.hypot(np.diff(xs), np.diff(ds)), 10e-6, rtol=0, atol=1e-15)
        assert np.allclose(np.diff(xs), 10e-6 * np.cos(a), rtol=0, atol=1e-15)
        assert np.allclose(np.diff(ds) / np.diff(xs), np.tan(a), rtol=1e-9)
    # continuous profile: across a joint the two half steps meet at the corner
    for f in range(3):
        a0, a1 = np.deg2rad(angles[f]), np.deg2rad(angles[f + 1])
        corner = np.array([x[128 * f + 127], d[128 * f + 127]]) + 5e-6 * np.array([np.cos(a0), np.sin(a0)])
        back = np.array([x[128 * f + 128], d[128 * f + 128]]) - 5e-6 * np.array([np.cos(a1), np.sin(a1)])
        assert np.allclose(corner, back, rtol=0, atol=1e-15)


def test_quadratic_arc_length():
    a = 100.0
    x, d = synth.quadratic_profile(1024, 10e-6, a)
    assert np.allclose(d, a * x * x, rtol=0, atol=0)
    assert np.all(np.diff(x) > 0) and np.allclose(x, -x[::-1], rtol=0, atol=1e-18)
    # arc length between neighbours by fine quadrature of sqrt(1 + (2 a x)^2)
    t = np.linspace(0.0, 1.0, 65)
    seg = x[:-1, None] + (x[1:] - x[:-1])[:, None] * t[None, :]
    arc = np.trapezoid(np.sqrt(1.0 + (2 * a * seg) ** 2), seg, axis=1)
    assert np.allclose(arc, 10e-6, rtol=1e-9, atol=0)
    # spacing in x1 is the pitch times cos of the local slope angle
    mid = 0.5 * (x[1:] + x[:-1])
    assert np.allclose(np.diff(x), 10e-6 / np.sqrt(1 + (2 * a * mid) ** 2), rtol=1e-6)


def test_line_configs():
    f = synth.line_config("facets_1d")
    q = synth.line_config("quadratic_1d")
    for w in (f, q):
        assert w.lam == 633e-9 and w.z0 == 1.0 and w.p2 == 10e-6 and w.m == 1024
        assert w.u.dtype == np.complex64 and np.all(w.u == 1)
    assert f.n == 512 and q.n == 1024
