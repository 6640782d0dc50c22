"""GPU parity: the HIP forward path against the FP64 CPU oracle.

Every case runs the whole path (geometry kernels, spreading, both FFT passes
with the fused deconvolution) through the C ABI and compares u2 with the
oracle's direct sum element by element.  Bars: relative L2 <= 1e-5 with FP32
FFT stages and <= 1e-4 with split-FP16 FFT stages, per evaluation set.
"""
import os

import numpy as np
import pytest

import synth
from gpu_util import eval_sets, gpu_forward, oracle_at, rel_l2, to_dev, torch_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-4}
ORACLE_THREADS = min(16, os.cpu_count() or 1)


def _oracle(w, ix, iy):
    import oracle
    return oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                         incident=w.incident, nthreads=ORACLE_THREADS)


def _full_grid(w):
    gx, gy = np.meshgrid(np.arange(w.mx), np.arange(w.my))
    return _oracle(w, gx.reshape(-1), gy.reshape(-1)).reshape(w.my, w.mx)


def _custom(nx, ny, pitch, jitter, mx, my, p2x, p2y, lam=532e-9, z0=0.1, amp=20e-6, period=0.8e-3,
            seed=4, incident="plane", tol=1e-5):
    rng = np.random.default_rng(seed)
    x, y = synth.jittered_grid(rng, nx, ny, pitch, jitter)
    d = synth.sinusoidal_relief(x, y, amp, period)
    u = synth.random_field(rng, nx, ny)
    return synth.Workload("custom", x, y, d, u, lam, z0, p2x, p2y, mx, my, tol, incident)


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_sinusoid_128_full_grid(fft):
    w = synth.config("sinusoid_128")
    got, info = gpu_forward(w, fft)
    want = _full_grid(w)
    err = rel_l2(got, want)
    print(f"sinusoid_128 {fft}: rel-L2 {err:.3e} (w={info['w']}, tiles={info['ntiles']})")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_ragged_nonsquare_no_incident(fft):
    """N = 37 x 53 (not a multiple of any block size), 64 x 32 output, p2x != p2y, u_I = 1."""
    w = _custom(37, 53, 8e-6, 2e-6, 64, 32, 9e-6, 7e-6, incident="none")
    got, _ = gpu_forward(w, fft)
    err = rel_l2(got, _full_grid(w))
    print(f"ragged {fft}: {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_wrapping_frequencies(fft):
    """Large destination pitch: x / (lambda r0) p2 spans more than one period and wraps."""
    w = _custom(96, 80, 8e-6, 2.4e-6, 128, 128, 80e-6, 70e-6, z0=0.1)
    k_t = w.p2x * np.abs(w.x).max() / (w.lam * (w.z0 - w.d.max()))
    assert k_t > 0.5   # cycles per destination pixel beyond half a period: both signs wrap
    got, _ = gpu_forward(w, fft)
    err = rel_l2(got, _full_grid(w))
    print(f"wrap {fft}: {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
def test_tolerance_sets_width(tol):
    """Every spreading width the tolerances select (w = ceil(log10(1/tol)) + 2, 3 .. 9):
    the requested accuracy, or the FP32 FFT's 1e-5 bar below it."""
    w = _custom(64, 64, 8e-6, 2e-6, 64, 64, 8e-6, 8e-6, tol=tol)
    got, info = gpu_forward(w, "fp32", tol=tol)
    assert info["w"] == round(-np.log10(tol)) + 2
    err = rel_l2(got, _full_grid(w))
    print(f"tol {tol}: w={info['w']} err {err:.3e}")
    assert err <= max(tol, 1e-5)


@pytest.mark.parametrize("fft,d0,incident", [("fp32", 0.0, "plane"), ("split_fp16", 0.0, "plane"),
                                             ("fp32", 12e-6, "none")])
def test_flat_grid_is_a_centred_dft(fft, d0, incident):
    """A flat surface (d1 = d0) on a regular grid with p2 = lambda r0 / (N p1), r0 = z0 - d0:
    the sum of Eq. (7) is a centred 2D DFT between the chirps (a closed form independent
    of the oracle); without the incident plane wave the constant phase exp(-i k d0) stays."""
    torch = torch_gpu()
    N, lam, z0, p1 = 64, 532e-9, 0.1, 8e-6
    r0 = z0 - d0
    p2 = lam * r0 / (N * p1)
    idx = np.arange(N) - N // 2
    yy, xx = np.meshgrid(idx * p1, idx * p1, indexing="ij")
    x, y = xx.reshape(-1), yy.reshape(-1)
    d = np.full_like(x, d0)
    rng = np.random.default_rng(5)
    u = (rng.standard_normal(N * N) + 1j * rng.standard_normal(N * N)).astype(np.complex64)
    w = synth.Workload("flat", x, y, d, u, lam, z0, p2, p2, N, N, incident=incident)
    got, _ = gpu_forward(w, fft)
    k = 2.0 * np.pi / lam
    c = u.astype(np.complex128).reshape(N, N) * np.exp(1j * k * (yy ** 2 + xx ** 2) / (2.0 * r0))
    if incident == "none":
        c = c * np.exp(-1j * k * d0)
    F = np.exp(-2j * np.pi * np.outer(idx, idx) / N)          # [m, i]: exp(-2 pi i m i / N)
    S = F @ c @ F.T                                            # rows: Y modes, columns: X modes
    X = p2 * idx
    chirp = np.exp(1j * k * (X[:, None] ** 2 + X[None, :] ** 2) / (2.0 * z0))
    want = np.exp(1j * k * z0) / (1j * lam * z0) * chirp * S
    err = rel_l2(got, want)
    print(f"flat grid {fft} d0={d0} {incident}: {err:.2e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_single_point(fft):
    """One point: u2 is a plane wave times the chirps, the same magnitude everywhere,
    so every destination pixel carries the kernel and deconvolution error alone."""
    w = _custom(1, 1, 8e-6, 3e-6, 32, 32, 8e-6, 8e-6)
    got, _ = gpu_forward(w, fft)
    err = rel_l2(got, _full_grid(w))
    print(f"single point {fft}: {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_hot_tile_all_points_in_one_cell_block(fft):
    """5000 points within a few fine cells: one tile holds every point."""
    rng = np.random.default_rng(9)
    n = 5000
    x = rng.uniform(-4e-6, 4e-6, n)
    y = rng.uniform(-4e-6, 4e-6, n)
    d = rng.uniform(0, 10e-6, n)
    u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    w = synth.Workload("hot", x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 64, 64)
    got, _ = gpu_forward(w, fft)
    err = rel_l2(got, _full_grid(w))
    print(f"hot tile {fft}: {err:.3e}")
    assert err <= TOL[fft]
    if fft != "fp32":
        return
    # slabs sized from these counts would not fit in 4 n slots: the plan keeps the
    # compact layout and re-bins by counting first, with the same result
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    xd, yd, dd, ud = to_dev(torch, w)
    plan = asf.Plan(xd, yd, dd, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)

    def status():   # the counters' copy of the latest binning
        return int(plan.workspace_view(plan.info()["off_status"], 1, torch.int32).item())

    first = plan.forward(ud).cpu().numpy()
    st0 = status()
    plan.setpts(xd, yd, dd)
    plan.status()
    again = plan.forward(ud).cpu().numpy()
    st1 = status()
    plan.close()
    assert st0 == 4 and st1 == 4
    assert np.array_equal(first, again)


def test_binning_layout_switches_with_crowding():
    """One plan re-binned between an even geometry (frequencies wrapping over the
    whole fine grid: every tile fits its first, uniform slab of 4 n / ntiles slots)
    and one with 40% of the points in one spot (four tiles overflow their slabs:
    the compact layout packs the bins).  The status word names the layout; a
    compact binning sizes new slabs from its tile counts, which the next binning
    of the same geometry fills in one pass, and which overflow again when the
    geometry changes back.  Every binning reproduces a fresh plan bit for bit and
    the oracle, and binnings of one geometry in either layout give the same forward and
    adjoint bit for bit (the slab and compact passes form the same records)."""
    torch = torch_gpu()
    import dataclasses
    import paper_1203_3583_amd as asf

    even = _custom(128, 128, 8e-6, 2e-6, 128, 128, 80e-6, 80e-6, seed=6)
    rng = np.random.default_rng(12)
    x, y = even.x.copy(), even.y.copy()
    crowd = rng.choice(even.n, size=(2 * even.n) // 5, replace=False)
    x[crowd] = rng.uniform(-2e-6, 2e-6, crowd.size)
    y[crowd] = rng.uniform(-2e-6, 2e-6, crowd.size)
    crowded = dataclasses.replace(even, name="crowded", x=x, y=y)

    xe, ye, de, u = to_dev(torch, even)
    xc, yc, dc, _ = to_dev(torch, crowded)
    plan = asf.Plan(xe, ye, de, even.lam, even.z0, even.p2x, even.p2y, even.mx, even.my)
    info = plan.info()
    assert crowd.size > info["slot_cap"] // info["ntiles"]   # crowded tiles cannot fit a slab
    copies = []
    g2 = torch.from_numpy(synth.random_field(np.random.default_rng(13), even.mx, even.my)).cuda()
    adjoints = []

    def run():
        # binnings alternate between two copies of the status word and cursors
        plan.status()
        at = plan.info()["off_status"]
        copies.append(at)
        adjoints.append(plan.adjoint(g2).cpu().numpy())
        return int(plan.workspace_view(at, 1, torch.int32).item()), plan.forward(u).cpu().numpy()

    seq = [run()]                                    # slabs
    for geo in ((xc, yc, dc), (xc, yc, dc), (xe, ye, de), (xe, ye, de)):
        plan.setpts(*geo)
        seq.append(run())
    assert copies[0] != copies[1] and copies[::2] == [copies[0]] * 3 and copies[1::2] == [copies[1]] * 2
    # uniform slabs hold; they overflow -> compact, new slabs fit (12); those hold;
    # sized for the crowd they overflow on the even geometry -> 12; resized, they hold
    assert [st for st, _ in seq] == [0, 12, 0, 12, 0]
    f_even, f_crowd = seq[0][1], seq[1][1]
    assert np.array_equal(seq[2][1], f_crowd)
    assert np.array_equal(seq[3][1], f_even) and np.array_equal(seq[4][1], f_even)
    # the adjoint carries each record's pre-phase in FP32 sums, unrounded: equal bits
    # mean both binning passes formed the same records
    assert np.array_equal(adjoints[2], adjoints[1])
    assert np.array_equal(adjoints[3], adjoints[0]) and np.array_equal(adjoints[4], adjoints[0])
    # the adjoint in the compact layout: <A u, g> = <u, A^H g>
    plan.setpts(xc, yc, dc)
    g = torch.from_numpy(synth.random_field(rng, even.mx, even.my)).cuda()
    au = plan.forward(u)
    ahg = plan.adjoint(g)
    lhs = torch.vdot(g.reshape(-1).to(torch.complex128), au.reshape(-1).to(torch.complex128)).item()
    rhs = torch.vdot(ahg.to(torch.complex128), u.to(torch.complex128)).item()
    plan.close()
    fresh_even, _ = gpu_forward(even)
    fresh_crowd, _ = gpu_forward(crowded)
    assert np.array_equal(f_even.astype(np.complex128), fresh_even)
    assert np.array_equal(f_crowd.astype(np.complex128), fresh_crowd)
    ix, iy = synth.sample_pixels(even.mx, even.my, 256, seed=3)
    assert rel_l2(f_crowd[iy, ix], _oracle(crowded, ix, iy)) <= 1e-5
    assert rel_l2(f_even[iy, ix], _oracle(even, ix, iy)) <= 1e-5
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


_ORACLE_CACHE = {}


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
@pytest.mark.parametrize("mx,my", [(16, 2048), (2048, 16), (32, 1024), (1024, 32), (64, 512), (512, 64),
                                   (16, 4096), (4096, 16)])
def test_every_transform_length(mx, my, fft):
    """Fine-grid lengths 32 .. 8192 along each axis (every length the two FFT passes
    are built for below the 16384 of the largest grid; lengths that are not powers of
    16 take a radix-2/4/8 first stage, 4096 the direct-I/O kernels), skinny grids whose
    32-cell side folds a padded tile onto itself, and 2999 scattered points whose
    frequencies wrap about one and a half periods: the whole output against the oracle."""
    key = (mx, my)
    if key not in _ORACLE_CACHE:
        rng = np.random.default_rng(mx * 7 + my)
        n = 2999
        x = rng.uniform(-5e-4, 5e-4, n)
        y = rng.uniform(-5e-4, 5e-4, n)
        d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
        u = (rng.uniform(0, 1, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))).astype(np.complex64)
        w = synth.Workload("lengths", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, mx, my, 1e-5, "plane")
        _ORACLE_CACHE[key] = (w, _full_grid(w))
    w, want = _ORACLE_CACHE[key]
    got, info = gpu_forward(w, fft)
    assert (info["nfx"], info["nfy"]) == (2 * mx, 2 * my)
    err = rel_l2(got, want)
    print(f"{mx} x {my} {fft}: rel-L2 {err:.3e}")
    assert err <= TOL[fft]


@pytest.mark.parametrize("fft", ["fp32", "split_fp16"])
def test_largest_destination_grid(fft):
    """The largest destination grid (8192 x 8192: a 16384^2 fine grid, 131072 tiles,
    16384-point transforms) with a million scattered points, on crops and random pixels."""
    rng = np.random.default_rng(21)
    n = 1 << 20
    x = rng.uniform(-5e-3, 5e-3, n)
    y = rng.uniform(-4e-3, 4e-3, n)
    d = synth.sinusoidal_relief(x, y, 25e-6, 0.7e-3)
    u = (rng.uniform(0, 1, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))).astype(np.complex64)
    w = synth.Workload("largest", x, y, d, u, 633e-9, 0.3, 4e-6, 4e-6, 8192, 8192, 1e-5, "plane")
    got, info = gpu_forward(w, fft)
    assert info["nfx"] == info["nfy"] == 16384 and info["ntiles"] == 131072
    for name, (ix, iy) in eval_sets(w, n_random=96, crop=6).items():
        err = rel_l2(got[iy, ix], _oracle(w, ix, iy))
        print(f"largest {fft} {name}: {err:.3e}")
        assert err <= TOL[fft], name


def test_linearity_and_repeat():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("cap_2048", side=256)
    x, y, d, u = to_dev(torch, w)
    rng = np.random.default_rng(2)
    v = torch.from_numpy(synth.random_field(rng, 256, 256)).cuda()
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    a, b = 0.7 - 0.2j, -0.3 + 1.1j
    fu = plan.forward(u).cpu().numpy()
    fv = plan.forward(v).cpu().numpy()
    fuv = plan.forward((a * u + b * v).to(torch.complex64)).cpu().numpy()
    fu2 = plan.forward(u).cpu().numpy()
    plan.close()
    assert rel_l2(fuv, a * fu + b * fv) <= 3e-6
    # the spread accumulates in integers, so a repeat is bitwise identical
    assert np.array_equal(fu2, fu)


@pytest.mark.parametrize("which", ["cap_256", "sinusoid_128", "bright"])
def test_point_order_does_not_change_the_output(which):
    """The same points in another order give bitwise the same u2: every decision of a
    spreading tile comes from maxima and integer counts and its sums are integers, so
    neither the input order nor the binning's record order (nor, for the 128^2 relief,
    how its crowded tiles are cut into slices) can change a bit; the FFT passes then
    see the same fine grid."""
    import dataclasses

    if which == "cap_256":
        w = synth.config("cap_2048", side=256)
    elif which == "sinusoid_128":
        w = synth.config("sinusoid_128")
    else:
        base = synth.config("cap_2048", side=256, out=256)
        rng = np.random.default_rng(17)
        u = (1e-4 * synth.random_field(rng, 256, 256)).astype(np.complex64)
        u[256 * 131 + 97] = 1.0
        w = dataclasses.replace(base, u=u)
    perm = np.random.default_rng(5).permutation(w.x.size)
    wp = dataclasses.replace(w, x=w.x[perm], y=w.y[perm], d=w.d[perm], u=w.u.reshape(-1)[perm])
    for fft in ("fp32", "split_fp16"):
        a, _ = gpu_forward(w, fft)
        b, _ = gpu_forward(wp, fft)
        assert np.array_equal(a, b), (which, fft)


def test_setpts_matches_new_plan():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w1 = synth.config("sinusoid_128", seed=0)
    w2 = synth.config("sinusoid_128", seed=3)
    x1, y1, d1, u1 = to_dev(torch, w1)
    x2, y2, d2, u2 = to_dev(torch, w2)
    plan = asf.Plan(x1, y1, d1, w1.lam, w1.z0, w1.p2x, w1.p2y, w1.mx, w1.my)
    plan.setpts(x2, y2, d2)
    plan.status()
    got = plan.forward(u2).cpu().numpy()
    plan.close()
    fresh, _ = gpu_forward(w2)
    assert rel_l2(got, fresh) <= 1e-6


def test_domain_errors_raise():
    torch = torch_gpu()
    import paper_1203_3583_amd as asf

    w = synth.config("sinusoid_128", side=16, out=16)
    x, y, d, _ = to_dev(torch, w)
    bad = d.clone()
    bad[5] = w.z0 + 1e-3              # r0 < 0
    with pytest.raises(asf.AsfError) as e:
        asf.Plan(x, y, bad, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    assert e.value.code == asf.asf.ASF_EDOMAIN
    xn = x.clone()
    xn[3] = float("nan")
    with pytest.raises(asf.AsfError) as e:
        asf.Plan(xn, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    assert e.value.code == asf.asf.ASF_EDOMAIN
    # a valid plan then a bad geometry through setpts: reported by status()
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    plan.setpts(x, y, bad)
    with pytest.raises(asf.AsfError) as e:
        plan.status()
    assert e.value.code == asf.asf.ASF_EDOMAIN
    plan.close()

