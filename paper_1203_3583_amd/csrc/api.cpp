// Host side of the library: parameter checks, workspace layout, FP64 tables and
// the extern "C" entry points declared in include/asf.h.
//
// Tables built here in FP64 and rounded once to complex64:
//   Dx[ix] = exp(i k z0) / (i lambda z0) * exp(i k X^2 / (2 z0)) / psi_hat_x(m),
//   Dy[iy] = exp(i k Y^2 / (2 z0)) / psi_hat_y(n),
// with X = p2x m, m = ix - mx/2 (Eq. (7)/(8): the post-phase of the destination,
// whose chirp uses z0 by the approximation of Eq. (6)), and psi_hat the Fourier
// transform of the spreading kernel at mode m on the fine grid, by
// Gauss-Legendre quadrature; twiddles exp(-2 pi i e / L) of both FFT lengths and
// the 16-point DFT roots.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "asf.h"
#include "asf_internal.h"
#include "plan_host.h"

using asf::FftShape;

namespace {

using namespace asf::host;

int hip_fail(hipError_t e, const char *what) {
    return fail(ASF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static_assert(asf::kSplitSlots == kSplitSlotsHost, "partial-tile slots");
static_assert(sizeof(Cf) == sizeof(float2), "host complex values are laid out like float2");

}  // namespace

struct asf_plan_s {
    Layout lay;
    asf_params prm;
    char *ws;
    asf::Binned bin;
    asf::GeoParams geo;
    asf::SpreadParams sp;
    FftShape sh1, sh2;
    int mid_panel;      // columns per panel of the column pass's output (sh1.batch or more)
    float2 *fine, *mid, *dx, *dy, *twx, *twy, *w16;
    int timing;
    bool count_first;   // bin with the compact layout directly (crowded last time)
    bool sparse;        // many tiles empty last time: leave them unwritten, the column pass reads zeros
    int copy;           // which copy of status and cursor the last binning used
    bool clear_both;    // clear both copies first (new plan, or a failed binning launch)
    uint32_t slots;     // workgroups resident at once (crowded tiles are cut against it); 0: never cut
    bool events;
    hipEvent_t ev[2 * asf::NSTAGES];
    bool recorded[asf::NSTAGES];
};

namespace {

int ensure_events(asf_plan_s *p) {
    if (p->events) return ASF_OK;
    for (int i = 0; i < 2 * asf::NSTAGES; ++i) {
        hipError_t e = hipEventCreate(&p->ev[i]);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(p->ev[j]);
            return hip_fail(e, "hipEventCreate");
        }
    }
    p->events = true;
    return ASF_OK;
}

struct StageMark {
    asf_plan_s *p;
    int stage;
    hipStream_t s;
    StageMark(asf_plan_s *p_, int st, hipStream_t s_) : p(p_), stage(st), s(s_) {
        if (p->timing) (void)hipEventRecord(p->ev[2 * stage], s);
    }
    ~StageMark() {
        if (p->timing) {
            (void)hipEventRecord(p->ev[2 * stage + 1], s);
            p->recorded[stage] = true;
        }
    }
};

// Point bin.status and bin.cursor at copy p->copy of the counters, and the
// next_ pointers at the other copy.
void bind_counters(asf_plan_s *p) {
    const Layout &L = p->lay;
    const size_t st[2] = {L.off_status, L.off_status2}, cu[2] = {L.off_cursor, L.off_cursor2};
    p->bin.status = reinterpret_cast<uint32_t *>(p->ws + st[p->copy]);
    p->bin.cursor = reinterpret_cast<uint32_t *>(p->ws + cu[p->copy]);
    p->bin.next_status = reinterpret_cast<uint32_t *>(p->ws + st[p->copy ^ 1]);
    p->bin.next_cursor = reinterpret_cast<uint32_t *>(p->ws + cu[p->copy ^ 1]);
}

int geometry_launches(asf_plan_s *p, const double *x, const double *y, const double *d, hipStream_t s) {
    hipError_t e;
    {
        StageMark m(p, asf::STAGE_BIN, s);
        if (p->clear_both) {
            e = asf::launch_bin_reset(p->bin, p->lay.ntiles, s);
            if (e != hipSuccess) return hip_fail(e, "bin_reset launch");
        }
        if (p->count_first) {
            e = asf::launch_bin_count(p->geo, p->bin, p->lay.n, x, y, d, s);
            if (e != hipSuccess) return hip_fail(e, "bin_count launch");
        } else {
            e = asf::launch_bin_fill(p->geo, p->bin, p->lay.n, x, y, d, s);
            if (e != hipSuccess) return hip_fail(e, "bin_fill launch");
        }
    }
    // compact layout: both kernels return at once when the slabs held
    {
        StageMark m(p, asf::STAGE_SCAN, s);
        e = asf::launch_bin_scan(p->bin, p->lay.ntiles, p->lay.ntx, p->slots, s);
        if (e != hipSuccess) return hip_fail(e, "bin_scan launch");
    }
    {
        StageMark m(p, asf::STAGE_SCATTER, s);
        e = asf::launch_bin_scatter(p->geo, p->bin, p->lay.n, p->lay.ntiles, x, y, d, s);
        if (e != hipSuccess) return hip_fail(e, "bin_scatter launch");
    }
    return ASF_OK;
}

// One binning, into the counters the previous binning's second pass cleared.
int run_geometry(asf_plan_s *p, const double *x, const double *y, const double *d, hipStream_t s) {
    p->copy ^= 1;
    bind_counters(p);
    const int rc = geometry_launches(p, x, y, d, s);
    p->clear_both = rc != ASF_OK;
    return rc;
}

int upload_tables(asf_plan_s *p, hipStream_t s) {
    const Layout &L = p->lay;
    const asf_params &q = p->prm;
    const double k = 2.0 * kPi / q.lambda;
    std::vector<float2> dx(L.mx), dy(L.my), w16(16);
    const std::vector<Cf> twx = stage_twiddles(L.nfx), twy = stage_twiddles(L.nfy);
    const std::vector<double> phx = psi_hat(L.mx / 2, L.nfx, L.w, L.beta);
    const std::vector<double> phy = psi_hat(L.my / 2, L.nfy, L.w, L.beta);
    // exp(i k z0) / (i lambda z0) = -i exp(i k z0) / (lambda z0)
    const double a0 = reduce(k * q.z0);
    const double c0r = std::sin(a0) / (q.lambda * q.z0), c0i = -std::cos(a0) / (q.lambda * q.z0);
    for (int ix = 0; ix < L.mx; ++ix) {
        const int m = ix - L.mx / 2;
        const double X = q.x0 + q.p2x * m;
        const double ch = reduce(k * X * X / (2.0 * q.z0));
        const double inv = 1.0 / phx[m < 0 ? -m : m];
        const double er = std::cos(ch) * inv, ei = std::sin(ch) * inv;
        dx[ix] = make_float2((float)(er * c0r - ei * c0i), (float)(er * c0i + ei * c0r));
    }
    for (int iy = 0; iy < L.my; ++iy) {
        const int n = iy - L.my / 2;
        const double Y = q.y0 + q.p2y * n;
        const double ch = reduce(k * Y * Y / (2.0 * q.z0));
        const double inv = 1.0 / phy[n < 0 ? -n : n];
        dy[iy] = make_float2((float)(std::cos(ch) * inv), (float)(std::sin(ch) * inv));
    }
    for (int e = 0; e < 16; ++e) {
        const double a = 2.0 * kPi * e / 16.0;
        w16[e] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    // the first slabs: uniform, a multiple of 16 slots but not of 256, so that the
    // tiles' slabs do not start at power-of-two strides (the workgroups spreading
    // neighbouring tiles would read the same memory channels)
    uint32_t cap = (uint32_t)(L.slot_cap / L.ntiles) & ~15u;
    if (cap >= 256 && cap % 256 == 0) cap -= 16;
    std::vector<uint2> slab(L.ntiles);
    for (int t = 0; t < L.ntiles; ++t) slab[t] = make_uint2((uint32_t)t * cap, cap);
    struct { void *dst; const void *src; size_t n; } copies[] = {
        {p->bin.slab, slab.data(), slab.size() * sizeof(uint2)},
        {p->dx, dx.data(), dx.size() * sizeof(float2)},
        {p->dy, dy.data(), dy.size() * sizeof(float2)},
        {p->twx, twx.data(), twx.size() * sizeof(Cf)},
        {p->twy, twy.data(), twy.size() * sizeof(Cf)},
        {p->w16, w16.data(), w16.size() * sizeof(float2)},
    };
    for (auto &c : copies) {
        hipError_t e = hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "table upload");
    }
    // the host vectors die here: wait for the copies
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ASF_OK;
}

int read_status(asf_plan_s *p, hipStream_t s) {
    uint32_t st = 0, empty = 0;
    hipError_t e = hipMemcpyAsync(&st, p->bin.status, sizeof st, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "status read");
    e = hipMemcpyAsync(&empty, p->bin.split_meta + 2, sizeof empty, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "empty-tile count read");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // a quarter of the tiles or more empty: the next transforms leave them unwritten
    // (spreading, the adjoint's column pass) and the forward's column pass reads them
    // as zeros (either form is exact for any geometry, the flags being rewritten by
    // every binning; this one saves the empty tiles' writes and reads)
    p->sparse = (uint64_t)empty * 4 >= (uint64_t)p->lay.ntiles;
    p->sp.skip_dead = p->sparse ? 1 : 0;
    // kStatusCompact and kStatusFits only describe the binned layout: the next
    // binning counts first if this one needed the compact layout, unless its
    // scan sized new slabs from the counts that fit in the slot arrays
    p->count_first = (st & asf::kStatusCompact) && !(st & asf::kStatusFits);
    if (st & asf::kStatusDomain)
        return fail(ASF_EDOMAIN, "some point has r0 = z0 - d1 <= 0 or a non-finite coordinate");
    if (st & asf::kStatusOverflow) return fail(ASF_EHIP, "internal error: tile bin overflow");
    return ASF_OK;
}

}  // namespace

extern "C" {

const char *asf_last_error(void) { return asf::host::last_error(); }

size_t asf_workspace_bytes(int64_t n_src, const asf_params *p) {
    Layout L;
    if (make_layout(n_src, p, L) != ASF_OK) return 0;
    return L.total;
}

int asf_plan(asf_plan_t *out, int64_t n_src, const double *x1, const double *y1, const double *d1,
             const asf_params *p, void *workspace, size_t ws_bytes, void *stream) {
    if (!out) return fail(ASF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!x1 || !y1 || !d1 || !workspace) return fail(ASF_EINVAL, "x1, y1, d1 and workspace must be non-NULL");
    Layout L;
    int rc = make_layout(n_src, p, L);
    if (rc) return rc;
    if (ws_bytes < L.total)
        return fail(ASF_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ASF_EINVAL, "workspace must be %zu-byte aligned", kAlign);

    asf_plan_s *pl = new (std::nothrow) asf_plan_s();
    if (!pl) return fail(ASF_EINVAL, "out of host memory");
    pl->lay = L;
    pl->prm = *p;
    pl->ws = static_cast<char *>(workspace);
    char *w = pl->ws;
    pl->copy = 1;   // the first binning takes copy 0
    pl->clear_both = true;
    bind_counters(pl);
    pl->bin.tile_start = reinterpret_cast<uint32_t *>(w + L.off_tile_start);
    pl->bin.key = reinterpret_cast<uint2 *>(w + L.off_cell);
    pl->bin.rec = reinterpret_cast<float4 *>(w + L.off_frac);
    pl->bin.slab = reinterpret_cast<uint2 *>(w + L.off_slab);
    pl->bin.slot_cap = (uint32_t)L.slot_cap;
    pl->bin.split = reinterpret_cast<uint32_t *>(w + L.off_split);
    pl->bin.split_meta = reinterpret_cast<uint32_t *>(w + L.off_split_meta);
    pl->bin.slot_owner = reinterpret_cast<uint32_t *>(w + L.off_slot_owner);
    pl->bin.live = reinterpret_cast<uint8_t *>(w + L.off_live);
    pl->bin.live_col = pl->bin.live + L.ntiles;
    pl->bin.combine = reinterpret_cast<uint32_t *>(w + L.off_combine);
    pl->bin.partial = reinterpret_cast<unsigned long long *>(w + L.off_partial);
    pl->fine = reinterpret_cast<float2 *>(w + L.off_fine);
    pl->mid = reinterpret_cast<float2 *>(w + L.off_mid);
    pl->dx = reinterpret_cast<float2 *>(w + L.off_dx);
    pl->dy = reinterpret_cast<float2 *>(w + L.off_dy);
    pl->twx = reinterpret_cast<float2 *>(w + L.off_twx);
    pl->twy = reinterpret_cast<float2 *>(w + L.off_twy);
    pl->w16 = reinterpret_cast<float2 *>(w + L.off_w16);

    const double k = 2.0 * kPi / p->lambda;
    pl->geo.k = k;
    pl->geo.inv_lambda = 1.0 / p->lambda;
    pl->geo.z0 = p->z0;
    pl->geo.p2x = p->p2x;
    pl->geo.p2y = p->p2y;
    pl->geo.x0 = p->x0;
    pl->geo.y0 = p->y0;
    pl->geo.nfx = L.nfx;
    pl->geo.nfy = L.nfy;
    pl->geo.w = L.w;
    pl->geo.log_tile_x = log2i(L.tile_x);
    pl->geo.log_tile_y = log2i(L.tile_y);
    pl->geo.ntx = L.ntx;
    pl->geo.nty = L.nty;
    pl->geo.plane = (p->flags & ASF_INCIDENT_NONE) ? 0 : 1;

    // FFT shapes: pass 1 holds `panel` adjacent columns of length nfy per workgroup
    // (the fine grid is stored in panels of that width), pass 2 whole rows
    const int lds_max = asf::fft_max_lds_bytes();
    const int panel = asf::fft_batch_pass1(L.nfy);
    pl->sh1.L = L.nfy;
    pl->sh1.batch = panel;
    pl->mid_panel = asf::fft_mid_panel(L.nfy);
    pl->sh2.L = L.nfx;
    pl->sh2.batch = asf::fft_batch_pass2(L.nfx);
    if (panel > L.tile_x || L.nfx % panel != 0 || L.my % pl->sh2.batch != 0 ||
        asf::fft_lds_bytes(L.nfy, panel) > (size_t)lds_max ||
        asf::fft_lds_bytes(L.nfx, pl->sh2.batch) > (size_t)lds_max) {
        delete pl;
        return fail(ASF_ESIZE, "FFT of %d x %d does not fit this device's LDS (%d bytes)", L.nfx, L.nfy, lds_max);
    }

    pl->sp.n = L.n;
    pl->sp.nfx = L.nfx;
    pl->sp.nfy = L.nfy;
    pl->sp.w = L.w;
    pl->sp.log_tile_x = log2i(L.tile_x);
    pl->sp.log_tile_y = log2i(L.tile_y);
    pl->sp.log_ntx = log2i(L.ntx);
    pl->sp.ntx = L.ntx;
    pl->sp.nty = L.nty;
    pl->sp.log_panel = log2i(panel);
    pl->sp.beta_log2e = (float)(L.beta * 1.4426950408889634);
    pl->sp.split = L.split ? 1 : 0;
    pl->sp.skip_dead = 0;
    pl->sparse = false;
    // three spreading workgroups fit a compute unit at once
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    pl->slots = L.split ? 3u * (uint32_t)cus : 0u;

    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = upload_tables(pl, s);
    if (!rc) rc = run_geometry(pl, x1, y1, d1, s);
    if (!rc) rc = read_status(pl, s);
    if (rc) {
        if (pl->events)
            for (int i = 0; i < 2 * asf::NSTAGES; ++i) (void)hipEventDestroy(pl->ev[i]);
        delete pl;
        return rc;
    }
    *out = pl;
    return ASF_OK;
}

int asf_setpts(asf_plan_t plan, const double *x1, const double *y1, const double *d1, void *stream) {
    if (!plan || !x1 || !y1 || !d1) return fail(ASF_EINVAL, "plan, x1, y1, d1 must be non-NULL");
    return run_geometry(plan, x1, y1, d1, static_cast<hipStream_t>(stream));
}

int asf_status(asf_plan_t plan, void *stream) {
    if (!plan) return fail(ASF_EINVAL, "plan is NULL");
    return read_status(plan, static_cast<hipStream_t>(stream));
}

namespace {

// The binning's per-tile flags for the column passes, when the plan leaves the tiles
// no record reaches unwritten.
asf::LiveTiles live_tiles(const asf_plan_s *p) {
    return asf::LiveTiles{p->sp.skip_dead ? p->bin.live : nullptr, p->bin.live_col, p->lay.ntx, p->lay.nty,
                          log2i(p->lay.tile_x), log2i(p->lay.tile_y)};
}

// Spread, column pass and row pass into u2; fine and mid are the fine grid and the
// column pass's output (the plan's workspace, or the static scratch).
int forward_into(asf_plan_t plan, const void *u1, void *u2, void *stream, int accumulate, float2 *fine,
                 float2 *mid) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    asf_plan_s *p = plan;
    const int split = (p->prm.flags & ASF_FFT_MASK) == ASF_FFT_SPLIT_FP16;
    hipError_t e;
    {
        StageMark m(p, asf::STAGE_SPREAD, s);
        e = asf::launch_spread(p->sp, p->bin, static_cast<const float2 *>(u1), fine, s);
        if (e != hipSuccess) return hip_fail(e, "spread launch");
    }
    {
        StageMark m(p, asf::STAGE_FFT1, s);
        e = asf::launch_fft_pass1(p->sh1, split, fine, mid, p->twy, p->w16, p->lay.nfx, p->lay.my,
                                  live_tiles(p), s);
        if (e != hipSuccess) return hip_fail(e, "fft pass 1 launch");
    }
    {
        StageMark m(p, asf::STAGE_FFT2, s);
        e = asf::launch_fft_pass2(p->sh2, log2i(p->mid_panel), split, mid, static_cast<float2 *>(u2),
                                  p->twx, p->w16, p->dx, p->dy, p->lay.mx, p->lay.my, accumulate,
                                  live_tiles(p), s);
        if (e != hipSuccess) return hip_fail(e, "fft pass 2 launch");
    }
    return ASF_OK;
}

int forward(asf_plan_t plan, const void *u1, void *u2, void *stream, int accumulate) {
    if (!plan || !u1 || !u2) return fail(ASF_EINVAL, "plan, u1, u2 must be non-NULL");
    return forward_into(plan, u1, u2, stream, accumulate, plan->fine, plan->mid);
}

}  // namespace

int asf_forward(asf_plan_t plan, const void *u1, void *u2, void *stream) {
    return forward(plan, u1, u2, stream, 0);
}

int asf_forward_add(asf_plan_t plan, const void *u1, void *u2, void *stream) {
    return forward(plan, u1, u2, stream, 1);
}

int asf_forward_static(asf_plan_t plan, const void *u1, void *u2, void *stream) {
    if (!plan || !u1 || !u2) return fail(ASF_EINVAL, "plan, u1, u2 must be non-NULL");
    const Layout &L = plan->lay;
    const size_t fine_bytes = align_up(sizeof(float2) * (size_t)L.nfx * L.nfy);
    const size_t mid_bytes = sizeof(float2) * (size_t)L.my * L.nfx;
    if (fine_bytes + mid_bytes > asf::kStaticScratchBytes)
        return fail(ASF_ESIZE, "the fine grid and column-pass output of a %d x %d destination need %zu bytes; "
                    "the static scratch holds %zu (destinations up to 1024 x 1024)", L.mx, L.my,
                    fine_bytes + mid_bytes, asf::kStaticScratchBytes);
    void *base = nullptr;
    hipError_t e = asf::static_scratch(&base);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    char *b = static_cast<char *>(base);
    return forward_into(plan, u1, u2, stream, 0, reinterpret_cast<float2 *>(b),
                        reinterpret_cast<float2 *>(b + fine_bytes));
}

int asf_adjoint(asf_plan_t plan, const void *g2, void *g1, void *stream) {
    if (!plan || !g2 || !g1) return fail(ASF_EINVAL, "plan, g2, g1 must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    asf_plan_s *p = plan;
    const int split = (p->prm.flags & ASF_FFT_MASK) == ASF_FFT_SPLIT_FP16;
    hipError_t e;
    {
        StageMark m(p, asf::STAGE_ADJ_FFT2, s);
        e = asf::launch_fft_adj_rows(p->lay.nfx, split, static_cast<const float2 *>(g2), p->mid, p->twx,
                                     p->w16, p->dx, p->dy, p->lay.mx, p->lay.my, live_tiles(p), s);
        if (e != hipSuccess) return hip_fail(e, "adjoint row pass launch");
    }
    {
        StageMark m(p, asf::STAGE_ADJ_FFT1, s);
        e = asf::launch_fft_adj_cols(p->lay.nfy, split, p->mid, p->fine, p->twy, p->w16, p->lay.nfx,
                                     p->lay.my, live_tiles(p), s);
        if (e != hipSuccess) return hip_fail(e, "adjoint column pass launch");
    }
    {
        StageMark m(p, asf::STAGE_INTERP, s);
        e = asf::launch_interp(p->sp, p->bin, p->fine, static_cast<float2 *>(g1), s);
        if (e != hipSuccess) return hip_fail(e, "interpolation launch");
    }
    return ASF_OK;
}

int asf_plan_info(asf_plan_t plan, asf_info *info) {
    if (!plan || !info) return fail(ASF_EINVAL, "plan and info must be non-NULL");
    const Layout &L = plan->lay;
    std::memset(info, 0, sizeof *info);
    info->n_src = L.n;
    info->mx = L.mx;
    info->my = L.my;
    info->nfx = L.nfx;
    info->nfy = L.nfy;
    info->w = L.w;
    info->beta = L.beta;
    info->tile_x = L.tile_x;
    info->tile_y = L.tile_y;
    info->ntiles = L.ntiles;
    info->slot_cap = L.slot_cap;
    info->col_batch = plan->sh1.batch;
    info->mid_panel = plan->mid_panel;
    info->flags = plan->prm.flags;
    info->off_status = plan->copy ? L.off_status2 : L.off_status;
    info->off_tile_start = L.off_tile_start;
    info->off_cell = L.off_cell;
    info->off_frac = L.off_frac;
    info->off_phase = L.off_phase;
    info->off_perm = L.off_perm;
    info->off_fine = L.off_fine;
    info->off_mid = L.off_mid;
    info->ws_bytes = L.total;
    info->off_cursor = plan->copy ? L.off_cursor2 : L.off_cursor;
    info->off_slab = L.off_slab;
    info->off_split = L.off_split;
    info->off_split_meta = L.off_split_meta;
    info->off_slot_owner = L.off_slot_owner;
    info->split_slots = plan->slots;
    info->off_live = L.off_live;
    info->skip_empty = plan->sparse ? 1u : 0u;
    return ASF_OK;
}

int asf_set_timing(asf_plan_t plan, int enable) {
    if (!plan) return fail(ASF_EINVAL, "plan is NULL");
    if (enable) {
        int rc = ensure_events(plan);
        if (rc) return rc;
    }
    plan->timing = enable ? 1 : 0;
    for (int i = 0; i < asf::NSTAGES; ++i) plan->recorded[i] = false;
    return ASF_OK;
}

int asf_stage_times(asf_plan_t plan, double *ms, int n) {
    if (!plan || !ms || n < 0) return fail(ASF_EINVAL, "plan and ms must be non-NULL");
    if (!plan->events) return fail(ASF_EINVAL, "timing was never enabled");
    int k = 0;
    for (; k < n && k < asf::NSTAGES; ++k) {
        ms[k] = -1.0;
        if (!plan->recorded[k]) continue;
        hipError_t e = hipEventSynchronize(plan->ev[2 * k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.f;
        e = hipEventElapsedTime(&t, plan->ev[2 * k], plan->ev[2 * k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ms[k] = t;
    }
    return k;
}

int asf_destroy(asf_plan_t plan) {
    if (!plan) return fail(ASF_EINVAL, "plan is NULL");
    if (plan->events)
        for (int i = 0; i < 2 * asf::NSTAGES; ++i) (void)hipEventDestroy(plan->ev[i]);
    delete plan;
    return ASF_OK;
}

}  // extern "C"

// ---- one-dimensional (line) plans ----------------------------------------------------
//
// Tables built in FP64 and rounded once to complex64:
//   D[ix] = exp(i k (z0 + X^2 / (2 z0))) / sqrt(i lambda z0) / psi_hat(k),  X = x0 + p2 k,
//   k = ix - m/2 (the 1D post-phase: the 2D prefactor 1/(i lambda z0) with one
//   axis integrated out, sqrt(i lambda z0) of the Fresnel chirp integral);
//   tw[e] = exp(-2 pi i e / nf), e < nf/2 (radix-2 stages).

struct asf_line_s {
    asf_line_params prm;
    asf::LineGeo geo;
    asf::LineBins bin;
    float2 *tw, *dd;
};

namespace {

int upload_line_tables(asf_line_s *p, const LineLayout &L, hipStream_t s) {
    const asf_line_params &q = p->prm;
    const double k = 2.0 * kPi / q.lambda;
    const std::vector<double> ph = psi_hat(L.m / 2, L.nf, L.w, L.beta);
    std::vector<float2> dd(L.m), tw(L.nf / 2);
    // 1 / sqrt(i lambda z0) = exp(-i pi/4) / sqrt(lambda z0)
    const double amp = 1.0 / std::sqrt(q.lambda * q.z0);
    for (int ix = 0; ix < L.m; ++ix) {
        const int m = ix - L.m / 2;
        const double X = q.x0 + q.p2 * m;
        const double a = reduce(reduce(k * q.z0) + reduce(k * X * X / (2.0 * q.z0)) - 0.25 * kPi);
        const double r = amp / ph[m < 0 ? -m : m];
        dd[ix] = make_float2((float)(r * std::cos(a)), (float)(r * std::sin(a)));
    }
    for (int e = 0; e < L.nf / 2; ++e) {
        const double a = 2.0 * kPi * e / L.nf;
        tw[e] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    hipError_t e = hipMemcpyAsync(p->dd, dd.data(), dd.size() * sizeof(float2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "line table upload");
    e = hipStreamSynchronize(s);   // the host vectors die here
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ASF_OK;
}

}  // namespace

extern "C" {

size_t asf_line_workspace_bytes(int64_t n_src, const asf_line_params *p) {
    LineLayout L;
    if (make_line_layout(n_src, p, L) != ASF_OK) return 0;
    return L.total;
}

int asf_line_plan(asf_line_t *out, int64_t n_src, const double *x1, const double *d1,
                  const asf_line_params *p, void *workspace, size_t ws_bytes, void *stream) {
    if (!out) return fail(ASF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!x1 || !d1 || !workspace) return fail(ASF_EINVAL, "x1, d1 and workspace must be non-NULL");
    LineLayout L;
    int rc = make_line_layout(n_src, p, L);
    if (rc) return rc;
    if (ws_bytes < L.total) return fail(ASF_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ASF_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    asf_line_s *pl = new (std::nothrow) asf_line_s();
    if (!pl) return fail(ASF_EINVAL, "out of host memory");
    pl->prm = *p;
    char *w = static_cast<char *>(workspace);
    pl->bin.status = reinterpret_cast<uint32_t *>(w + L.off_status);
    pl->bin.first = reinterpret_cast<uint32_t *>(w + L.off_first);
    pl->bin.perm = reinterpret_cast<uint32_t *>(w + L.off_perm);
    pl->bin.cell = reinterpret_cast<uint32_t *>(w + L.off_cell);
    pl->bin.coef = reinterpret_cast<float2 *>(w + L.off_coef);
    pl->tw = reinterpret_cast<float2 *>(w + L.off_tw);
    pl->dd = reinterpret_cast<float2 *>(w + L.off_dd);
    pl->geo.inv_lambda = 1.0 / p->lambda;
    pl->geo.z0 = p->z0;
    pl->geo.p2 = p->p2;
    pl->geo.x0 = p->x0;
    pl->geo.n = L.n;
    pl->geo.m = L.m;
    pl->geo.nf = L.nf;
    pl->geo.log_nf = log2i(L.nf);
    pl->geo.w = L.w;
    pl->geo.plane = (p->flags & ASF_INCIDENT_NONE) ? 0 : 1;
    pl->geo.beta = L.beta;

    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = upload_line_tables(pl, L, s);
    if (!rc) {
        // the status word starts at zero: a one-word copy from host memory, then the setup kernel
        static const uint32_t zero = 0;
        hipError_t e = hipMemcpyAsync(pl->bin.status, &zero, sizeof zero, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = asf::launch_line_setup(pl->geo, pl->bin, x1, d1, s);
        if (e != hipSuccess) rc = hip_fail(e, "line setup");
    }
    if (!rc) {
        uint32_t st = 0;
        hipError_t e = hipMemcpyAsync(&st, pl->bin.status, sizeof st, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "line status read");
        else if (st & 1u) rc = fail(ASF_EDOMAIN, "some point has r0 = z0 - d1 <= 0 or a non-finite coordinate");
    }
    if (rc) {
        delete pl;
        return rc;
    }
    *out = pl;
    return ASF_OK;
}

int asf_line_forward(asf_line_t plan, int32_t batch, const void *u1, void *u2, void *stream) {
    if (!plan || !u1 || !u2) return fail(ASF_EINVAL, "plan, u1, u2 must be non-NULL");
    if (batch < 1) return fail(ASF_EINVAL, "batch must be >= 1, got %d", batch);
    hipError_t e = asf::launch_line_forward(plan->geo, plan->bin, plan->tw, plan->dd, batch,
                                            static_cast<const float2 *>(u1), static_cast<float2 *>(u2),
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "line forward launch");
    return ASF_OK;
}

int asf_line_destroy(asf_line_t plan) {
    if (!plan) return fail(ASF_EINVAL, "plan is NULL");
    delete plan;
    return ASF_OK;
}

}  // extern "C"
