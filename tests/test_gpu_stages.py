"""Stage-by-stage checks of the HIP forward path, each stage against a host FP64
model fed with the device's own input to that stage:

  a1/a2  binning: every point's first footprint cell (exact), offsets (FP32 of the
         FP64 value), pre-phase exp(i phi) (FP32 sincos), and the tile bins (exact
         multiset of (tile, point) pairs, in both the slab and the compact layout);
  a3     spreading: the fine grid against a direct FP64 sum of the exponential-of-
         semicircle footprints of the device's records;
  a4/a5  column pass: the kept modes against numpy's FFT of the device's fine grid;
  a6     row pass: u2 against numpy's FFT of the device's column-pass output times
         the deconvolution and destination phase of Eq. (8), tables built here in FP64;
  adjoint: its row pass, column pass and interpolation, each the same way.

The host models restate the definitions (Eqs. (7)-(9), the kernel and its Fourier
transform); they share no code with the kernels.
"""
import numpy as np
import pytest

import synth
from gpu_util import rel_l2, to_dev, torch_gpu

pytestmark = pytest.mark.gpu


def _even():
    """128^2 points whose frequencies wrap over the whole fine grid (slab layout)."""
    rng = np.random.default_rng(21)
    x, y = synth.jittered_grid(rng, 128, 128, 8e-6, 2e-6)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    u = synth.random_field(rng, 128, 128).reshape(-1)
    return synth.Workload("even", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, 128, 128)


def _crowded():
    """The C1 relief: points in 15% of each axis' period (compact layout)."""
    return synth.config("sinusoid_128")


def _sparse():
    """A 2048^2 destination (4096^2 fine grid, 8192 tiles, several per resident
    workgroup) with 24 clusters of 1500 points, each cluster within a few tiles:
    a workgroup walks many tiles, most of them empty, between the non-empty ones."""
    rng = np.random.default_rng(31)
    centres = rng.uniform(-5e-3, 5e-3, size=(24, 2))
    x = (centres[:, 0, None] + rng.uniform(-4e-6, 4e-6, size=(24, 1500))).reshape(-1)
    y = (centres[:, 1, None] + rng.uniform(-4e-6, 4e-6, size=(24, 1500))).reshape(-1)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    n = x.size
    u = (rng.uniform(0, 1, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))).astype(np.complex64)
    return synth.Workload("sparse", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, 2048, 2048)


def _many_hot():
    """48 clusters of 12,000 points, each within a cell or two of a 2048^2 fine grid: some
    hundred crowded tiles whose 1024-record slices would need more than the 512 partial
    slots, so the cut lengthens its slices."""
    rng = np.random.default_rng(41)
    centres = rng.uniform(-5e-3, 5e-3, size=(48, 2))
    x = (centres[:, 0, None] + rng.uniform(-0.1e-6, 0.1e-6, size=(48, 12000))).reshape(-1)
    y = (centres[:, 1, None] + rng.uniform(-0.1e-6, 0.1e-6, size=(48, 12000))).reshape(-1)
    d = synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3)
    n = x.size
    u = (rng.uniform(0, 1, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))).astype(np.complex64)
    return synth.Workload("many_hot", x, y, d, u, 532e-9, 0.1, 80e-6, 80e-6, 1024, 1024)


def _bright():
    """One bright point over 256^2 points 1e4 times weaker (the tiles holding it take
    the split sums with 42-bit terms)."""
    base = synth.config("cap_2048", side=256, out=256)
    rng = np.random.default_rng(17)
    u = (1e-4 * synth.random_field(rng, 256, 256)).astype(np.complex64)
    u[256 * 131 + 97] = 1.0
    return synth.Workload("bright", base.x, base.y, base.d, u, base.lam, base.z0, base.p2x, base.p2y,
                          base.mx, base.my)


def _plan(torch, w, fft="fp32"):
    import paper_1203_3583_amd as asf

    x, y, d, u = to_dev(torch, w)
    plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, fft=fft)
    return plan, u


def _view(torch, plan, off, count, dtype):
    return plan.workspace_view(off, count, dtype).cpu().numpy()


def _host_points(w, nf_x, nf_y, wid):
    """First footprint cell, offsets and exp(i phi) per point in FP64 (Eqs. (7)-(9)),
    in the same operation order as a plain evaluation of the definitions."""
    s = (1.0 / w.lam) / (w.z0 - w.d)                       # 1 / (lambda r0)

    def axis(xi, nf):
        fr = xi - np.floor(xi)
        g = fr * nf
        g = np.where(g >= nf, g - nf, g)
        c = np.ceil(g - 0.5 * wid).astype(np.int64)
        off = g - c - 0.5 * (wid - 1)
        return np.where(c < 0, c + nf, c), off

    cx, ox = axis(w.p2x * w.x * s, nf_x)
    cy, oy = axis(w.p2y * w.y * s, nf_y)
    rev = 0.5 * s * (w.x * w.x + w.y * w.y)                 # plane-wave incidence
    t = rev - np.rint(rev)
    return cx, cy, ox, oy, np.exp(2j * np.pi * t)


def _host_bins(cx, cy, wid, nf_x, nf_y, tx, ty, ntx):
    """(tile, point) pairs: a point is listed in every tile its w x w footprint touches."""
    pairs = []
    lx = (cx + wid - 1) % nf_x
    ly = (cy + wid - 1) % nf_y
    for j in range(cx.size):
        xs = {cx[j] // tx, lx[j] // tx}
        ys = {cy[j] // ty, ly[j] // ty}
        for a in ys:
            for b in xs:
                pairs.append((int(a * ntx + b), j))
    return sorted(pairs)


def _device_bins(torch, plan, info):
    st = int(_view(torch, plan, info["off_status"], 1, torch.int32)[0])
    T = info["ntiles"]
    if st & 4:   # compact
        start = _view(torch, plan, info["off_tile_start"], T + 1, torch.int32).astype(np.int64)
        ranges = [(start[t], start[t + 1]) for t in range(T)]
    else:
        cnt = _view(torch, plan, info["off_cursor"], T, torch.int32).astype(np.int64)
        slab = _view(torch, plan, info["off_slab"], 2 * T, torch.int32).astype(np.int64).reshape(T, 2)
        ranges = [(slab[t, 0], slab[t, 0] + min(cnt[t], slab[t, 1])) for t in range(T)]
    return st, ranges


def _hot():
    """5000 points on a 64 x 64 grid: few tiles, each holding thousands of records."""
    rng = np.random.default_rng(9)
    n = 5000
    x = rng.uniform(-4e-6, 4e-6, n)
    y = rng.uniform(-4e-6, 4e-6, n)
    d = rng.uniform(0, 10e-6, n)
    u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    return synth.Workload("hot", x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 64, 64)


# (workload, binnings of the same points, status of the last one): uniform slabs;
# overflow into the compact layout whose counts size new slabs (12 = compact + fit);
# those sized slabs filled by the looping slab pass (0); a tile too crowded for sized
# slabs (4 = compact, no fit), after which the plan counts first (4)
BINNINGS = {"even": (_even, 1, 0), "crowded": (_crowded, 1, 12), "crowded_sized": (_crowded, 2, 0),
            "hot": (_hot, 1, 4), "hot_count_first": (_hot, 2, 4)}


@pytest.mark.parametrize("which", list(BINNINGS))
def test_binning_matches_host(which):
    """Every binning path lists exactly the host's (tile, point) pairs, each record
    holding the host's cell and FP32 offsets and a pre-phase within FP32 rounding."""
    torch = torch_gpu()
    make, times, want_st = BINNINGS[which]
    w = make()
    plan, _ = _plan(torch, w)
    for _ in range(times - 1):
        plan.status()
        plan.setpts(*to_dev(torch, w)[:3])
    plan.status()
    info = plan.info()
    nfx, nfy, wid = info["nfx"], info["nfy"], info["w"]
    tx, ty = info["tile_x"], info["tile_y"]
    st, ranges = _device_bins(torch, plan, info)
    cap = info["slot_cap"]
    # records: (cell, perm) as 8-byte words, (frac, phase) as 16-byte words
    key = _view(torch, plan, info["off_cell"], 2 * cap, torch.int32).reshape(-1, 2)
    assert info["off_perm"] == info["off_cell"] + 4 and info["off_phase"] == info["off_frac"] + 8
    rec = _view(torch, plan, info["off_frac"], 4 * cap, torch.float32).reshape(-1, 4)
    cell = key[:, 0].view(np.uint32)
    perm = key[:, 1].astype(np.int64)
    frac, phase = rec[:, 0:2], rec[:, 2:4]
    plan.close()
    assert st == want_st

    cx, cy, ox, oy, ph = _host_points(w, nfx, nfy, wid)
    got = sorted((t, int(perm[s])) for t, (a, b) in enumerate(ranges) for s in range(a, b))
    want = _host_bins(cx, cy, wid, nfx, nfy, tx, ty, nfx // tx)
    assert got == want                                      # exact tile lists
    slots = np.concatenate([np.arange(a, b) for a, b in ranges])
    j = perm[slots]
    assert np.array_equal(cell[slots] & 0xFFFF, cx[j]) and np.array_equal(cell[slots] >> 16, cy[j])
    assert np.array_equal(frac[slots, 0], ox[j].astype(np.float32))
    assert np.array_equal(frac[slots, 1], oy[j].astype(np.float32))
    dev = phase[slots, 0] + 1j * phase[slots, 1]
    assert np.max(np.abs(dev - ph[j])) <= 4e-7             # FP32 phase (<= 2e-7 rad) and sincos


def _host_split(counts, slots):
    """The cut of crowded tiles, by its rule: with R records and `slots` workgroups
    resident at once, a tile of more than max(2048, 2 ceil(R / slots)) records takes
    min(32, ceil(count / len)) slices (cut only if that is 2 or more), len =
    max(1024, ceil(R / slots)) doubled until all cut tiles need at most 512 slots."""
    r = int(counts.sum())
    load = -(-r // slots)
    thr = max(2048, 2 * load)
    if counts.max() <= thr:
        return None, np.zeros_like(counts), None
    ln = max(1024, load)
    while True:
        ns = np.where(counts > thr, np.minimum(32, -(-counts // ln)), 0)
        ns[ns < 2] = 0
        if ns.sum() <= 512:
            return thr, ns, ln
        ln *= 2


@pytest.mark.parametrize("which", ["even", "crowded", "hot", "sparse", "many_hot"])
def test_split_plan_matches_rule(which):
    """The binning's scan cuts exactly the tiles its rule names, into that many
    slices, with partial-tile slots handed out in tile order and every slot's
    owner recorded."""
    torch = torch_gpu()
    w = {"even": _even, "crowded": _crowded, "hot": _hot, "sparse": _sparse, "many_hot": _many_hot}[which]()
    plan, _ = _plan(torch, w)
    plan.status()
    info = plan.info()
    T = info["ntiles"]
    _, ranges = _device_bins(torch, plan, info)
    meta = _view(torch, plan, info["off_split_meta"], 2, torch.int32).view(np.uint32)
    split = _view(torch, plan, info["off_split"], T, torch.int32).view(np.uint32)
    owner = _view(torch, plan, info["off_slot_owner"], 512, torch.int32).view(np.uint32)
    plan.close()
    counts = np.array([b - a for a, b in ranges], dtype=np.int64)
    slots = info["split_slots"]
    assert slots > 0
    thr, ns, ln = _host_split(counts, slots)
    print(f"split {which}: slots {slots}, largest tile {counts.max()}, threshold {thr}, "
          f"cut tiles {int((ns > 0).sum())}, partial slots {int(ns.sum())}")
    if thr is None:
        assert meta[1] == 0 and meta[0] == 0xFFFFFFFF
        return
    assert meta[0] == thr and meta[1] == ns.sum()
    at = 0
    for t in np.flatnonzero(counts > thr):
        if ns[t] == 0:
            assert split[t] == 0
            continue
        assert split[t] == (at << 8 | ns[t])
        for q in range(ns[t]):
            assert owner[at + q] == (t << 8 | q)
        at += ns[t]
    if which in ("crowded", "hot", "many_hot"):
        assert (ns > 0).any()   # these geometries are cut
    if which == "many_hot":
        assert ln > 1024         # and this one needed longer slices


def test_cut_tiles_are_deterministic():
    """Spreading a cut geometry twice gives bitwise the same fine grid (the partial
    tiles are summed in slice order whichever slice finishes last)."""
    torch = torch_gpu()
    w = _hot()
    plan, u = _plan(torch, w)
    info = plan.info()
    grids = []
    for _ in range(3):
        plan.forward(u)
        torch.cuda.synchronize()
        grids.append(_view(torch, plan, info["off_fine"], 2 * info["nfx"] * info["nfy"], torch.int32))
    plan.close()
    assert np.array_equal(grids[0], grids[1]) and np.array_equal(grids[0], grids[2])


def _psi(z, wid, beta):
    a = 1.0 - (2.0 * z / wid) ** 2
    return np.where(a >= 0.0, np.exp(beta * (np.sqrt(np.maximum(a, 0.0)) - 1.0)), 0.0)


def _live_cells(torch, plan, info, flags=False):
    """[gy, gx] True in the tiles the binning flags as reached by some record (flags), or,
    by default, in the tiles the transforms write: those, in the plan's sparse form, else
    all (grids too small for cut tiles have no flags)."""
    if not flags and not plan.info()["skip_empty"]:
        return np.ones((info["nfy"], info["nfx"]), dtype=bool)
    tx_n, ty_n = info["nfx"] // info["tile_x"], info["nfy"] // info["tile_y"]
    live = _view(torch, plan, info["off_live"], tx_n * ty_n, torch.uint8).reshape(ty_n, tx_n)
    return np.repeat(np.repeat(live != 0, info["tile_y"], axis=0), info["tile_x"], axis=1)


def _live_columns(torch, plan, info, flags=False):
    """[gx] True in the tile columns holding a tile some record reaches (the others are
    zeros, which the column passes skip and the row passes do not touch in mid in the
    plan's sparse form); by default all columns outside the sparse form."""
    if not flags and not plan.info()["skip_empty"]:
        return np.ones(info["nfx"], dtype=bool)
    tx_n = info["nfx"] // info["tile_x"]
    col = _view(torch, plan, info["off_live"] + info["ntiles"], tx_n, torch.uint8)
    return np.repeat(col != 0, info["tile_x"])


def _fine_natural(torch, plan, info, after_forward=True):
    """The fine grid as [gy, gx].  After a forward, tiles no record reaches may have
    been left unwritten (holding whatever was there); they are taken as zeros, as the
    column pass reads them."""
    nfx, nfy, C = info["nfx"], info["nfy"], info["col_batch"]
    raw = _view(torch, plan, info["off_fine"], 2 * nfx * nfy, torch.float32)
    # (re, im) pairs as complex: unwritten tiles may hold any bits, signalling NaNs too
    with np.errstate(invalid="ignore"):
        v = np.ascontiguousarray(raw).view(np.complex64).astype(np.complex128)
    # element (gx, gy) at ((gx / C) nfy + gy) C + gx % C -> [gy, gx]
    fine = v.reshape(nfx // C, nfy, C).transpose(1, 0, 2).reshape(nfy, nfx)
    if after_forward:
        fine = np.where(_live_cells(torch, plan, info), fine, 0.0)
    return fine


@pytest.mark.parametrize("which", ["even", "crowded", "hot", "sparse", "bright", "many_hot"])
def test_spread_matches_host_sum(which):
    """Even points (slab layout), the crowded relief (compact layout), a small grid
    whose tiles hold thousands of records (start histogram, record reloads), a large
    grid of mostly empty tiles (each workgroup walks many tiles) and a bright point
    over a weak field (split sums with 42-bit terms).  The bar is relative to the
    whole grid; for the bright point the weak field's own part of the grid (the cells
    the bright point does not reach) is also checked against its own norm."""
    torch = torch_gpu()
    w = {"even": _even, "crowded": _crowded, "hot": _hot, "sparse": _sparse, "bright": _bright,
         "many_hot": _many_hot}[which]()
    plan, u = _plan(torch, w)
    plan.forward(u)
    torch.cuda.synchronize()
    info = plan.info()
    fine = _fine_natural(torch, plan, info)
    live = _live_cells(torch, plan, info)
    plan.close()
    nfx, nfy, wid, beta = info["nfx"], info["nfy"], info["w"], info["beta"]
    cx, cy, ox, oy, ph = _host_points(w, nfx, nfy, wid)
    c = w.u.astype(np.complex128).reshape(-1) * ph
    want = np.zeros((nfy, nfx), dtype=np.complex128)
    a = np.arange(wid)
    kx = _psi(a[None, :] - 0.5 * (wid - 1) - ox[:, None], wid, beta)   # [n, w]
    ky = _psi(a[None, :] - 0.5 * (wid - 1) - oy[:, None], wid, beta)
    ix = (cx[:, None] + a[None, :]) % nfx
    iy = (cy[:, None] + a[None, :]) % nfy
    for r in range(wid):
        for q in range(wid):
            np.add.at(want, (iy[:, r], ix[:, q]), c * ky[:, r] * kx[:, q])
    err = rel_l2(fine, want)
    print(f"spread {which}: rel-L2 {err:.2e}")
    assert err <= 2e-6
    # the tiles flagged as reached by no record receive nothing
    assert not want[~live].any()
    if which == "bright":
        # the weak field alone, away from the bright point's footprint: 42-bit terms
        # keep its rounding far below the 2^-21 of the bright point's amplitude
        j = int(np.argmax(np.abs(w.u)))
        far = np.ones_like(want, dtype=bool)
        for r in range(wid):
            far[iy[j, r], ix[j, :]] = False
        err_w = rel_l2(fine[far], want[far])
        print(f"spread bright, weak cells: rel-L2 {err_w:.2e}")
        assert err_w <= 2e-6


def _psi_hat(m, nf, wid, beta):
    xq, wq = np.polynomial.legendre.leggauss(200)
    es = np.exp(beta * (np.sqrt(1.0 - xq * xq) - 1.0))
    return 0.5 * wid * np.sum(wq * es * np.cos(np.pi * np.outer(m, xq) * wid / nf), axis=1)


def test_unwritten_tiles_follow_the_geometry():
    """A plan re-binned between a geometry whose frequencies cover the whole fine grid
    and one that leaves nearly every tile empty.  Every binning flags the tiles some
    record reaches; the empty-tile count read with the status picks the form of the
    next transforms: every tile written (empty ones as zeros), or only the flagged
    ones, the forward's column pass reading the rest as zeros -- while the fine grid
    there still holds the previous geometry's sums.  Both forms give the same forward
    and adjoint bit for bit, whichever geometry they meet, and equal a fresh plan's."""
    torch = torch_gpu()
    import dataclasses
    import paper_1203_3583_amd as asf

    sp = _sparse()
    rng = np.random.default_rng(51)
    x, y = rng.uniform(-6e-4, 6e-4, sp.n), rng.uniform(-6e-4, 6e-4, sp.n)
    dense = dataclasses.replace(sp, name="dense", x=x, y=y, d=synth.sinusoidal_relief(x, y, 20e-6, 0.8e-3))
    geo_s, geo_d = to_dev(torch, sp)[:3], to_dev(torch, dense)[:3]
    u = to_dev(torch, sp)[3]
    g2 = torch.from_numpy(synth.random_field(rng, sp.mx, sp.my)).cuda()

    def fresh(geo):
        plan = asf.Plan(*geo, sp.lam, sp.z0, sp.p2x, sp.p2y, sp.mx, sp.my)
        out = plan.forward(u).cpu().numpy(), plan.adjoint(g2).cpu().numpy()
        plan.close()
        return out

    want_s, want_d = fresh(geo_s), fresh(geo_d)
    plan = asf.Plan(*geo_s, sp.lam, sp.z0, sp.p2x, sp.p2y, sp.mx, sp.my)
    info = plan.info()

    def step():
        out = plan.forward(u).cpu().numpy()
        live = _live_cells(torch, plan, info, flags=True)
        fine = _fine_natural(torch, plan, info, after_forward=False)
        # the flags name exactly the tiles some record reaches
        _, ranges = _device_bins(torch, plan, plan.info())   # the binning's copy of the counters
        tx_n, ty_n = info["nfx"] // info["tile_x"], info["nfy"] // info["tile_y"]
        reached = np.array([b > a for a, b in ranges]).reshape(ty_n, tx_n)
        flags = _view(torch, plan, info["off_live"], tx_n * ty_n, torch.uint8).reshape(ty_n, tx_n)
        assert np.array_equal(flags, reached.astype(np.uint8))
        adj = plan.adjoint(g2).cpu().numpy()
        return out, adj, live, fine

    def same(got, want):
        return np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])

    out, adj, live, fine = step()   # sparse geometry, flagged form (from the plan's own status read)
    print(f"sparse: {int((~live).sum())} of {live.size} cells in empty tiles")
    assert (~live).sum() * 4 >= live.size and same((out, adj), want_s)
    assert plan.info()["skip_empty"] == 1
    plan.setpts(*geo_d)             # dense geometry, still the flagged form
    out, adj, live, fine = step()
    assert same((out, adj), want_d)
    plan.status()                   # dense: every tile written
    assert plan.info()["skip_empty"] == 0
    out, adj, live, fine = step()
    assert (~live).sum() * 4 < live.size and same((out, adj), want_d)
    plan.setpts(*geo_s)             # sparse geometry, every tile written: zeros in the empty ones
    out, adj, live, fine = step()
    assert same((out, adj), want_s)
    assert not fine[~live].any()
    plan.setpts(*geo_d)
    plan.status()
    plan.forward(u)                 # the whole fine grid holds the dense sums
    plan.setpts(*geo_s)
    plan.status()                   # sparse again: the empty tiles keep those sums
    assert plan.info()["skip_empty"] == 1
    out, adj, live, fine = step()
    plan.close()
    assert np.abs(fine[~live]).max() > 0     # stale sums really are there
    assert same((out, adj), want_s)


def _skinny(my):
    """The even points onto a 16-column destination my rows high: columns of 2 my
    points, whose column pass writes mid in panels wider than its one column."""
    import dataclasses
    return dataclasses.replace(_even(), name=f"skinny_{my}", mx=16, my=my)


@pytest.mark.parametrize("which", ["even", "crowded", "skinny_2048", "skinny_4096"])
@pytest.mark.parametrize("fft,bar", [("fp32", 2e-6), ("split_fp16", 1e-4)])
def test_fft_passes_match_numpy(fft, bar, which):
    """Both passes, each from the device's own input to it.  In the crowded relief most
    tiles are empty: their cells are read as zeros, the columns of tile columns with no
    reached tile are neither transformed nor read (zeros in the host's check).  The
    skinny grids have 4096- and 8192-point columns: one column per column-pass
    workgroup, mid in panels of two and four columns."""
    torch = torch_gpu()
    w = {"even": _even, "crowded": _crowded, "skinny_2048": lambda: _skinny(2048),
         "skinny_4096": lambda: _skinny(4096)}[which]()
    plan, u = _plan(torch, w, fft)
    u2 = plan.forward(u).cpu().numpy().astype(np.complex128)
    info = plan.info()
    fine = _fine_natural(torch, plan, info)
    cols = _live_columns(torch, plan, info)
    if which.startswith("skinny"):
        assert info["col_batch"] == 1 and info["mid_panel"] == {2048: 2, 4096: 4}[w.my]
    if which == "even":
        assert cols.all()
    elif which == "crowded":
        assert info["skip_empty"] == 1 and not cols.all()
    nfx, nfy, mx, my, P = info["nfx"], info["nfy"], w.mx, w.my, info["mid_panel"]
    raw = _view(torch, plan, info["off_mid"], 2 * my * nfx, torch.float32)
    plan.close()
    mid = (raw[0::2] + 1j * raw[1::2]).astype(np.complex128)
    mid = mid.reshape(nfx // P, my, P).transpose(1, 0, 2).reshape(my, nfx)   # [ky, x]
    mid = np.where(cols[None, :], mid, 0.0)
    # column pass: exp(-i) DFT along y of the device's fine grid, modes -my/2 .. my/2 - 1
    ky = (np.arange(my) - my // 2) % nfy
    want_mid = np.fft.fft(fine, axis=0)[ky, :]
    assert not want_mid[:, ~cols].any()
    e1 = rel_l2(mid, want_mid)
    # row pass: DFT along x of the device's mid, times 1/psi-hat, the destination chirp
    # and exp(i k z0) / (i lambda z0) (Eq. (8))
    kx = (np.arange(mx) - mx // 2) % nfx
    spec = np.fft.fft(mid, axis=1)[:, kx]
    k = 2.0 * np.pi / w.lam
    m = np.arange(mx) - mx // 2
    n = np.arange(my) - my // 2
    X, Y = w.p2x * m, w.p2y * n
    dx = np.exp(1j * k * X * X / (2.0 * w.z0)) / _psi_hat(np.abs(m), nfx, info["w"], info["beta"])
    dy = np.exp(1j * k * Y * Y / (2.0 * w.z0)) / _psi_hat(np.abs(n), nfy, info["w"], info["beta"])
    pre = np.exp(1j * k * w.z0) / (1j * w.lam * w.z0)
    want_u2 = pre * spec * dy[:, None] * dx[None, :]
    e2 = rel_l2(u2, want_u2)
    print(f"{fft}: column pass {e1:.2e}, row pass {e2:.2e}")
    assert e1 <= bar and e2 <= bar


@pytest.mark.parametrize("which", ["even", "crowded"])
@pytest.mark.parametrize("fft,bar", [("fp32", 2e-6), ("split_fp16", 1e-4)])
def test_adjoint_stages_match_host(fft, bar, which):
    """The adjoint's three stages, each from the device's own input to it: the row pass
    (g2 times conj(Dx Dy), zero-padded, exp(+i) DFT), the column pass (exp(+i) DFT of the
    kept rows) and the interpolation (conj(exp(i phi)) times the footprint sum).  The
    column pass is checked in the tiles some record reaches: in the crowded relief most
    tiles are empty and left unwritten, and no footprint reaches them."""
    torch = torch_gpu()
    w = {"even": _even, "crowded": _crowded}[which]()
    plan, u = _plan(torch, w, fft)
    info = plan.info()
    nfx, nfy, mx, my, C = info["nfx"], info["nfy"], w.mx, w.my, info["col_batch"]
    wid, beta = info["w"], info["beta"]
    rng = np.random.default_rng(8)
    g2 = torch.from_numpy(synth.random_field(rng, mx, my).reshape(my, mx)).cuda()
    g1 = plan.adjoint(g2).cpu().numpy().astype(np.complex128)
    torch.cuda.synchronize()
    raw = _view(torch, plan, info["off_mid"], 2 * my * nfx, torch.float32)
    mid = (raw[0::2] + 1j * raw[1::2]).astype(np.complex128).reshape(my, nfx)   # row-major
    fine = _fine_natural(torch, plan, info, after_forward=False)
    live = _live_cells(torch, plan, info)
    cols = _live_columns(torch, plan, info)
    plan.close()
    mid = np.where(cols[None, :], mid, 0.0)   # columns the column pass does not need
    k = 2.0 * np.pi / w.lam
    m = np.arange(mx) - mx // 2
    n = np.arange(my) - my // 2
    X, Y = w.p2x * m, w.p2y * n
    dx = np.exp(1j * k * X * X / (2.0 * w.z0)) / _psi_hat(np.abs(m), nfx, wid, beta)
    dy = np.exp(1j * k * Y * Y / (2.0 * w.z0)) / _psi_hat(np.abs(n), nfy, wid, beta)
    pre = np.exp(1j * k * w.z0) / (1j * w.lam * w.z0)
    g = g2.cpu().numpy().astype(np.complex128) * np.conj(pre * dy[:, None] * dx[None, :])
    pad = np.zeros((my, nfx), dtype=np.complex128)
    pad[:, m % nfx] = g
    want_mid = np.fft.ifft(pad, axis=1) * nfx                 # exp(+i), unnormalised
    e1 = rel_l2(mid[:, cols], want_mid[:, cols])
    padc = np.zeros((nfy, nfx), dtype=np.complex128)
    padc[n % nfy, :] = mid
    want_fine = np.fft.ifft(padc, axis=0) * nfy
    e2 = rel_l2(fine[live], want_fine[live])
    if which == "even":
        assert live.all() and cols.all()
    # interpolation from the device's fine grid, exact kernel values
    cx, cy, ox, oy, ph = _host_points(w, nfx, nfy, wid)
    a = np.arange(wid)
    kx = _psi(a[None, :] - 0.5 * (wid - 1) - ox[:, None], wid, beta)
    ky = _psi(a[None, :] - 0.5 * (wid - 1) - oy[:, None], wid, beta)
    ix = (cx[:, None] + a[None, :]) % nfx
    iy = (cy[:, None] + a[None, :]) % nfy
    acc = np.zeros(w.n, dtype=np.complex128)
    for r in range(wid):
        for q in range(wid):
            acc += fine[iy[:, r], ix[:, q]] * ky[:, r] * kx[:, q]
    want_g1 = np.conj(ph) * acc
    e3 = rel_l2(g1, want_g1)
    print(f"adjoint {fft}: rows {e1:.2e}, columns {e2:.2e}, interpolation {e3:.2e}")
    assert e1 <= bar and e2 <= bar and e3 <= 2e-6
