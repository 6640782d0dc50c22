// Geometry stage on gfx950: the FP64 pre-phase of Eq. (8) and the per-point
// frequencies of Eq. (9) (Sec. 2), and binning of the points into fine-grid
// tiles for the spreading kernel.
//
// For point j with r0 = z0 - d1 (Eq. (4)):
//   phi_j  = k (-d_j + |x_j|^2 / (2 r0_j)) + arg u_I,j        (pre-phase, Eq. (7)/(8))
//            - k (x_j x0 + y_j y0) / r0_j                  (destination window centred at x0, y0)
//   xi_j   = p2 x_j / (lambda r0_j)                           (cycles per destination pixel)
// With the normal plane wave u_I = exp(i k d1) the -k d1 term and the incident
// phase cancel exactly, so the kernel forms phi = k |x|^2 / (2 r0) directly and
// never builds the ~1e4 rad intermediate.  The phase is formed in FP64 in
// revolutions, phi / (2 pi) = |x|^2 s / 2 (- d / lambda without the plane
// wave), with s = 1 / (lambda r0) the same factor the frequencies use; its
// integer part is removed exactly in FP64 and only the remainder in
// [-1/2, 1/2] revolutions is rounded to FP32 for sincos(pi t) (phase error
// below 2e-7 rad, whatever the size of phi).  xi is wrapped to [0, 1)
// (exp(-2 pi i m xi) is 1-periodic in xi for integer m) and scaled to the fine
// grid, g = xi * nf.
// The footprint of the spreading kernel starts at cell l0 = ceil(g - w/2); the
// FP32 offset g - l0 - (w-1)/2 lies in (-1/2, 1/2], so its rounding error is at
// most 2^-26 cell however large the phase was.
//
// Binning: each point is listed once in every tile its w x w footprint touches
// (1, 2 or 4 tiles), so the spreading kernel can own its tile outright and write
// it with plain stores.  One pass bins the points into slabs of slots, one per
// tile: a per-tile cursor hands out the slots and counts the records.  The
// first slabs are uniform (the workspace holds 4 slots per point, so a slab has
// 4 n / ntiles), which suits points that cover the fine grid evenly.  If some
// tile receives more records than its slab (points crowded into part of the
// grid), the compact layout is built instead: an exclusive scan of the per-tile
// counts, then a second pass that packs the records in tile order.  The scan
// and that pass are always launched and return at once when the slabs held, so
// the host never waits for the decision (the scan first cuts crowded tiles into
// slices of records for the spreading kernel, from the counts of either layout:
// a tile far above the mean load of a resident workgroup would otherwise run
// alone long after the rest of the grid).  The scan also sizes new slabs from
// the counts (a quarter and 16 slots of headroom each) for the next binning; a
// plan whose last synchronised binning needed the compact layout bins into
// those if they fit, and otherwise counts first (a lighter pass than a slab
// pass it would waste).  The status word and the cursors exist twice: a
// binning uses one copy while its second pass clears the other for the next
// binning, so no launch of its own clears the counters.  Slot reservation aggregates per wavefront: the lanes
// are grouped by tile without memory traffic, then one lane per group issues
// the atomic -- all groups' atomics in the same instruction, so a wave waits for
// one round trip rather than one per tile.
#include "asf_internal.h"

namespace asf {
namespace {

struct PointTiles {
    int n;        // tiles touched (0 if the point is invalid)
    int key[4];   // tile indices ty * ntx + tx
    int l0x, l0y; // first footprint cell, wrapped into the fine grid
    float fx, fy; // offsets in (-1/2, 1/2]
    double s;     // 1 / (lambda r0)
};

// The counting and the scattering kernel must derive identical cells from the
// same point, so no FMA contraction is allowed to differ between them.
__device__ inline void axis_cell(double xi, int nf, int w, int &l0, float &off) {
#pragma clang fp contract(off)
    double fr = xi - floor(xi);             // [0, 1]
    double g = fr * (double)nf;
    if (g >= (double)nf) g -= (double)nf;   // fr rounded up to 1
    int c = (int)ceil(g - 0.5 * (double)w);
    off = (float)(g - (double)c - 0.5 * (double)(w - 1));
    if (c < 0) c += nf;
    l0 = c;
}

__device__ inline int axis_tiles(int l0, int nf, int w, int log_tile, int *t) {
    int last = l0 + w - 1;
    if (last >= nf) last -= nf;
    t[0] = l0 >> log_tile;
    t[1] = last >> log_tile;
    return t[1] != t[0] ? 2 : 1;
}

__device__ inline PointTiles point_tiles(const GeoParams &g, double x, double y, double d) {
#pragma clang fp contract(off)
    PointTiles p;
    p.n = 0;
    p.l0x = p.l0y = 0;
    p.fx = p.fy = 0.f;
    p.s = 0.0;
    const double r0 = g.z0 - d;
    if (!(r0 > 0.0) || !isfinite(x) || !isfinite(y) || !isfinite(d)) return p;
    p.s = g.inv_lambda / r0;
    axis_cell(g.p2x * x * p.s, g.nfx, g.w, p.l0x, p.fx);
    axis_cell(g.p2y * y * p.s, g.nfy, g.w, p.l0y, p.fy);
    int tx[2], ty[2];
    const int nx = axis_tiles(p.l0x, g.nfx, g.w, g.log_tile_x, tx);
    const int ny = axis_tiles(p.l0y, g.nfy, g.w, g.log_tile_y, ty);
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b) p.key[p.n++] = ty[a] * g.ntx + tx[b];
    return p;
}

// The pre-phase of Eq. (8) in revolutions, reduced to [-1/2, 1/2]: phi / (2 pi) =
// k (|x|^2 / (2 r0) [- d]) / (2 pi) = |x|^2 s / 2 [- d / lambda], and for an off-axis
// window -k (x x0 + y y0) / r0 = -2 pi (x x0 + y y0) s.  FP64 with contraction off, so
// that every binning pass forms the same bits for a point; the integer part is removed
// exactly, then one rounding to FP32.
__device__ inline float prephase_revolutions(const GeoParams &g, double x, double y, double d, double s) {
#pragma clang fp contract(off)
    double rev = 0.5 * s * (x * x + y * y);
    if (!g.plane) rev -= d * g.inv_lambda;
    rev -= (x * g.x0 + y * g.y0) * s;
    return (float)(rev - rint(rev));
}

// Group the active lanes of a wave by key (no memory traffic).  Every lane gets
// the lane id of its group's leader (the lowest lane with that key) and its
// rank within the group; leaders also get the group size.  All lanes of the
// wave must call this together.
struct WaveGroup {
    int leader;
    uint32_t rank;
    uint32_t size;   // meaningful on leaders
};

__device__ inline WaveGroup wave_group(int key, bool active) {
    const int lane = __lane_id();
    uint64_t todo = __ballot(active);
    uint64_t mine = 0ull;   // the lanes of this lane's group (0 if inactive)
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        // leader is wave-uniform: read its key with v_readlane, not an LDS permute
        const int lkey = __builtin_amdgcn_readlane(key, leader);
        const bool in = active && key == lkey;
        const uint64_t mask = __ballot(in);
        if (in) mine = mask;
        todo &= ~mask;
    }
    // rank: group lanes below this one (v_mbcnt); the leader is the lowest of them
    WaveGroup g;
    g.rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mine >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mine, 0u));
    g.size = (uint32_t)__popcll(mine);
    g.leader = mine ? __ffsll((unsigned long long)mine) - 1 : lane;
    return g;
}

// Both copies of the counters (at plan creation, and after a failed launch), and
// the slice counters of cut tiles
__global__ void __launch_bounds__(256) bin_reset_kernel(Binned b, int ntiles) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntiles) b.cursor[i] = b.next_cursor[i] = 0u;
    if (i < kSplitSlots) b.combine[i] = 0u;
    if (i == 0) {
        b.status[0] = b.next_status[0] = 0u;
        b.split_meta[0] = kNoSplit;
        b.split_meta[1] = 0u;
    }
}

constexpr int kGeoThreads = 256;
// points per thread, their loads in flight together: the counting pass is light
// on registers and takes four; the binning passes take two, which keeps them at
// 70-85 VGPRs (measured on the 2048^2 cap: 0.088 ms with four, 0.074 ms with two)
constexpr int kCountPoints = 4;
constexpr int kBinPoints = 2;
// workgroups of the compact layout's second pass, which loops over the point
// blocks: one round of the whole chip at its 5 waves per SIMD, and when no slab
// overflowed the launch costs only these returning at once
constexpr int kFallbackBlocks = 1280;

// point j of this thread's k-th batch in block blk (P batches per block):
// consecutive lanes take consecutive points
template <int P = kBinPoints>
__device__ inline int64_t geo_index(int64_t blk, int k) {
    return (blk * P + k) * kGeoThreads + threadIdx.x;
}

// Bin the points of block blk.  SLAB: reserve slots in the tiles' slabs; a
// record past its slab's end is counted but not written, and selects the
// compact layout.  Compact: the cursors start at the tiles' scanned offsets.
// All lanes of the wave must call this together.
template <bool SLAB>
__device__ inline void bin_block(const GeoParams &g, const Binned &b, int64_t n, int64_t blk,
                                 const double *__restrict__ x, const double *__restrict__ y,
                                 const double *__restrict__ d) {
    double xv[kBinPoints], yv[kBinPoints], dv[kBinPoints];
    // kStatusCompact is known set (wave-uniform): a crowded geometry overflows in
    // nearly every wave, and one status word taking an atomic from each of them
    // serialises the pass (4.2 ms instead of 0.6 ms on the 4096^2 relief)
    bool compact_known = false;
#pragma unroll
    for (int k = 0; k < kBinPoints; ++k) {
        const int64_t j = geo_index(blk, k);
        const bool in = j < n;
        xv[k] = in ? x[j] : 0.0;
        yv[k] = in ? y[j] : 0.0;
        dv[k] = in ? d[j] : 0.0;
    }
    PointTiles p[kBinPoints];
    WaveGroup grp[kBinPoints][4];
    uint32_t base[kBinPoints][4];
    // per replica: its tile's slab (slab layout) or end of its scanned range
    // (compact layout), loaded unconditionally (tile 0 for absent replicas) so that
    // the loads are in flight while the lanes are grouped
    uint2 lim[kBinPoints][4];
#pragma unroll
    for (int k = 0; k < kBinPoints; ++k) {
        p[k].n = 0;
        const bool in = geo_index(blk, k) < n;
        if (in) p[k] = point_tiles(g, xv[k], yv[k], dv[k]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int key = r < p[k].n ? p[k].key[r] : 0;
            lim[k][r] = SLAB ? b.slab[key] : make_uint2(0u, b.tile_start[key + 1]);
        }
        // one flag per wave holding invalid points
        if (SLAB && __ballot(in && p[k].n == 0) != 0ull && __lane_id() == 0) atomicOr(b.status, kStatusDomain);
        // group the replica keys, then let the leaders reserve their groups'
        // slots; the atomics of all batches and replicas are in flight at once
#pragma unroll
        for (int r = 0; r < 4; ++r) grp[k][r] = wave_group(r < p[k].n ? p[k].key[r] : 0, r < p[k].n);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            base[k][r] = (r < p[k].n && grp[k][r].leader == __lane_id())
                             ? atomicAdd(&b.cursor[p[k].key[r]], grp[k][r].size) : 0u;
    }
    // every replica's slot within its tile: the group leader's reservation plus the
    // lane's rank (all shuffles issued together)
    uint32_t pos[kBinPoints][4];
#pragma unroll
    for (int k = 0; k < kBinPoints; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) pos[k][r] = __shfl(base[k][r], grp[k][r].leader) + grp[k][r].rank;
#pragma unroll
    for (int k = 0; k < kBinPoints; ++k) {
        float2 ph = make_float2(0.f, 0.f);
        if (p[k].n > 0) {
            float sn, cs;
            sincospif(2.f * prephase_revolutions(g, xv[k], yv[k], dv[k], p[k].s), &sn, &cs);
            ph = make_float2(cs, sn);
        }
        const uint32_t cell = (uint32_t)p[k].l0x | ((uint32_t)p[k].l0y << 16);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool act = r < p[k].n;
            uint32_t slot;
            bool ok;
            if (SLAB) {
                slot = lim[k][r].x + pos[k][r];
                ok = pos[k][r] < lim[k][r].y;
                // at most one flag per wave, none once the bit is seen set: a crowded
                // tile can overflow by millions of records
                if (!compact_known && __ballot(act && !ok) != 0ull) {
                    compact_known = true;
                    if (__lane_id() == 0 &&
                        !(__hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStatusCompact))
                        atomicOr(b.status, kStatusCompact);
                }
            } else {
                slot = pos[k][r];
                ok = act && slot < lim[k][r].y;
                if (act && !ok) atomicOr(b.status, kStatusOverflow);
            }
            if (act && ok) {
                b.key[slot] = make_uint2(cell, (uint32_t)geo_index(blk, k));
                b.rec[slot] = make_float4(p[k].fx, p[k].fy, ph.x, ph.y);
            }
        }
    }
}

// Point blocks in a scattered order: the i-th workgroup of a pass takes block
// (i stride) mod nblk, stride coprime to nblk and near 0.618 nblk, so that the
// workgroups in flight together hold points from all over the surface.  Points
// that are neighbours in the caller's order tend to be neighbours in frequency,
// and consecutive blocks would have every wave in flight reserving slots in the
// same few tiles' cursors, each returning atomic waiting behind the others
// (4096^2 relief: 0.30 ms in consecutive order with a loop of 1280 workgroups,
// 0.21 ms scattered).
__device__ inline int64_t scattered_block(int64_t i, int64_t stride, int64_t nblk) {
    return (i * stride) % nblk;
}

__global__ void __launch_bounds__(kGeoThreads) bin_fill_kernel(GeoParams g, Binned b, int64_t n,
                                                               const double *__restrict__ x,
                                                               const double *__restrict__ y,
                                                               const double *__restrict__ d,
                                                               int64_t stride) {
    const int64_t per = (int64_t)kGeoThreads * kBinPoints;
    const int64_t nblk = (n + per - 1) / per;
    bin_block<true>(g, b, n, scattered_block(blockIdx.x, stride, nblk), x, y, d);
}

// Count-first binning (the compact layout without the slab pass): records per
// tile, one non-returning atomic per distinct tile per wave and replica.
__global__ void __launch_bounds__(kGeoThreads) bin_count_kernel(GeoParams g, Binned b, int64_t n,
                                                                const double *__restrict__ x,
                                                                const double *__restrict__ y,
                                                                const double *__restrict__ d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(b.status, kStatusCompact);
    double xv[kCountPoints], yv[kCountPoints], dv[kCountPoints];
#pragma unroll
    for (int k = 0; k < kCountPoints; ++k) {
        const int64_t j = geo_index<kCountPoints>(blockIdx.x, k);
        const bool in = j < n;
        xv[k] = in ? x[j] : 0.0;
        yv[k] = in ? y[j] : 0.0;
        dv[k] = in ? d[j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kCountPoints; ++k) {
        PointTiles p;
        p.n = 0;
        const bool in = geo_index<kCountPoints>(blockIdx.x, k) < n;
        if (in) p = point_tiles(g, xv[k], yv[k], dv[k]);
        if (__ballot(in && p.n == 0) != 0ull && __lane_id() == 0) atomicOr(b.status, kStatusDomain);
        for (int r = 0; r < 4; ++r) {
            const bool act = r < p.n;
            const WaveGroup grp = wave_group(act ? p.key[r] : 0, act);
            if (act && grp.leader == __lane_id()) atomicAdd(&b.cursor[p.key[r]], grp.size);
        }
    }
}

// Compact layout: exclusive scan of the per-tile counts by one workgroup of
// 1024 threads, in chunks of 8192 tiles: each thread loads 8 consecutive counts
// at once, the thread sums are scanned within waves by shuffles and across the
// 16 waves through LDS, and a running carry links the chunks.  A second scan
// sizes slabs for the next binning from the same counts, each with a quarter
// and 16 slots of headroom (a multiple of 16 slots); if they fit in the slot
// arrays they are written and kStatusFits is set.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;

__device__ inline uint32_t slab_want(uint32_t count) {
    const uint64_t w = ((uint64_t)count + (count >> 2) + 31u) & ~(uint64_t)15u;
    return w < 0xfffffff0ull ? (uint32_t)w : 0xfffffff0u;
}

// Exclusive scan of f(t) over the tiles in 64-bit sums; calls put(t, start,
// value) for each tile and returns the total.  Every thread of the block must
// call it.
template <class F, class P>
__device__ inline uint64_t block_scan(const Binned &b, int ntiles, uint64_t *wsum, F f, P put) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint64_t carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads * kScanPer) {
        const int lo = base + t * kScanPer;
        uint32_t v[kScanPer];
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = lo + k < ntiles ? f(lo + k) : 0u;
            s += v[k];
        }
        uint64_t inc = s;   // inclusive scan within the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t u = __shfl_up(inc, off);
            if (lane >= off) inc += u;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        if (wave == 0) {
            uint64_t u = lane < kScanThreads / 64 ? wsum[lane] : 0u;
#pragma unroll
            for (int off = 1; off < kScanThreads / 64; off <<= 1) {
                const uint64_t q = __shfl_up(u, off);
                if (lane >= off) u += q;
            }
            if (lane < kScanThreads / 64) wsum[lane] = u;   // inclusive totals of waves 0..lane
        }
        __syncthreads();
        uint64_t run = carry + (wave ? wsum[wave - 1] : 0u) + inc - s;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (lo + k < ntiles) put(lo + k, run, v[k]);
            run += v[k];
        }
        carry += wsum[kScanThreads / 64 - 1];
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    return carry;
}

// Slices of crowded tiles, from the binning's record counts.  The spreading and
// interpolation launches have ntiles + kSplitSlots workgroups; a tile is cut when
// its count exceeds max(kSplitMinRecords, 2 R / slots) -- R records over the
// slots workgroups resident at once -- into ceil(count / len) slices (at most
// kSplitMaxSlices) of len = max(kSliceMinRecords, R / slots) records.  Cut tiles
// take partial-tile slots in tile order; if they would need more than kSplitSlots,
// len doubles until they do not.
template <class C>
__device__ inline void split_plan(const Binned &b, int ntiles, int ntx, uint32_t slots, uint64_t *wsum,
                                  uint32_t *wmax, uint32_t *wempty, uint8_t *lcol, C count) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (slots == 0) {   // grids whose tiles are never cut (nor left unwritten: no flags)
        if (t == 0) {
            b.split_meta[0] = kNoSplit;
            b.split_meta[1] = 0u;
            b.split_meta[2] = 0u;
        }
        return;
    }
    // per tile column: whether some tile of it holds a record (plain stores of 1)
    for (int i = t; i < ntx; i += kScanThreads) lcol[i] = 0;
    __syncthreads();
    uint64_t r = 0;
    uint32_t most = 0, empty = 0;
    const bool compact = (b.status[0] & kStatusCompact) != 0u;
    // each tile's flag (some record reaches it) is stored one round late, after the
    // next round's loads are issued, so that waiting for those loads does not also
    // wait for these stores
    uint32_t flags = 0;
    int flag_base = -1;
    auto store_flags = [&]() {
        if (flag_base < 0) return;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = flag_base + k * kScanThreads + t;
            if (i < ntiles) b.live[i] = (uint8_t)((flags >> k) & 1u);
        }
    };
    for (int base = 0; base < ntiles; base += kScanThreads * kScanPer) {
        // kScanPer tiles' counts and slab sizes in flight (indices clamped so that
        // no load waits on a branch)
        uint32_t cur[kScanPer], cap[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = min(base + k * kScanThreads + t, ntiles - 1);
            cur[k] = b.cursor[i];
            cap[k] = b.slab[i].y;
        }
        store_flags();
        flags = 0;
        flag_base = base;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const bool in = base + k * kScanThreads + t < ntiles;
            const uint32_t c = in ? (compact ? cur[k] : min(cur[k], cap[k])) : 0u;
            r += c;
            most = max(most, c);
            empty += (in && c == 0u) ? 1u : 0u;
            flags |= (c != 0u ? 1u : 0u) << k;
            if (c != 0u) lcol[(base + k * kScanThreads + t) & (ntx - 1)] = 1;
        }
    }
    store_flags();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        r += __shfl_xor(r, off);
        most = max(most, (uint32_t)__shfl_xor((int)most, off));
        empty += (uint32_t)__shfl_xor((int)empty, off);
    }
    if (lane == 0) {
        wsum[wave] = r;
        wmax[wave] = most;
        wempty[wave] = empty;
    }
    __syncthreads();
    r = 0;
    most = 0;
    empty = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        r += wsum[k];
        most = max(most, wmax[k]);
        empty += wempty[k];
    }
    // tiles no record reaches, which the spreading and the adjoint's column pass may
    // leave unwritten (read by the host with the status, to choose that form for the
    // plan's next transforms)
    if (t == 0) b.split_meta[2] = empty;
    for (int i = t; i < ntx; i += kScanThreads) b.live_col[i] = lcol[i];
    __syncthreads();   // wsum is reused by the scans
    const uint64_t load = (r + slots - 1) / slots;
    const uint64_t thr64 = max((uint64_t)kSplitMinRecords, 2 * load);
    if (most <= thr64) {
        if (t == 0) {
            b.split_meta[0] = kNoSplit;
            b.split_meta[1] = 0u;
        }
        return;
    }
    const uint32_t thr = (uint32_t)thr64;   // < most
    uint64_t len = max((uint64_t)kSliceMinRecords, load);
    for (;;) {
        const auto slices = [&](int i) -> uint32_t {
            const uint32_t c = count(i);
            if (c <= thr) return 0u;
            const uint64_t ns = min((uint64_t)kSplitMaxSlices, (c + len - 1) / len);
            return ns >= 2 ? (uint32_t)ns : 0u;
        };
        const uint64_t used = block_scan(b, ntiles, wsum, slices, [&](int i, uint64_t at, uint32_t ns) {
            if (ns == 0) {
                if (count(i) > thr) b.split[i] = 0u;   // crowded, but one slice
                return;
            }
            if (at + ns > (uint64_t)kSplitSlots) return;   // redone with longer slices
            b.split[i] = (uint32_t)at << 8 | ns;
            for (uint32_t q = 0; q < ns; ++q) b.slot_owner[at + q] = (uint32_t)i << 8 | q;
        });
        if (used <= (uint64_t)kSplitSlots) {
            if (t == 0) {
                b.split_meta[0] = thr;
                b.split_meta[1] = (uint32_t)used;
            }
            return;
        }
        len *= 2;
    }
}

__global__ void __launch_bounds__(kScanThreads) bin_scan_kernel(Binned b, int ntiles, int ntx, uint32_t slots) {
    __shared__ uint64_t wsum[kScanThreads / 64];
    __shared__ uint32_t wmax[kScanThreads / 64], wempty[kScanThreads / 64];
    __shared__ uint8_t lcol[kMaxTileCols];
    const bool compact = (b.status[0] & kStatusCompact) != 0u;
    // record counts: the compact layout's counting pass, or the slabs' cursors
    // (past a full slab a cursor keeps counting records that were not written)
    split_plan(b, ntiles, ntx, slots, wsum, wmax, wempty, lcol, [&](int i) -> uint32_t {
        return compact ? b.cursor[i] : min(b.cursor[i], b.slab[i].y);
    });
    if (!compact) return;   // every slab held its tile
    // slabs for the next binning, written only if they fit (the total is uniform
    // over the block), then the compact layout itself (slot counts never exceed
    // 4 n < 2^32), which rewrites the counts as insertion cursors
    const auto want = [&](int i) { return slab_want(b.cursor[i]); };
    const uint64_t need = block_scan(b, ntiles, wsum, want, [](int, uint64_t, uint32_t) {});
    const bool fits = need <= (uint64_t)b.slot_cap;
    if (fits)
        block_scan(b, ntiles, wsum, want,
                   [&](int t, uint64_t start, uint32_t v) { b.slab[t] = make_uint2((uint32_t)start, v); });
    const uint64_t total = block_scan(
        b, ntiles, wsum, [&](int i) { return b.cursor[i]; },
        [&](int t, uint64_t start, uint32_t) {
            b.tile_start[t] = (uint32_t)start;
            b.cursor[t] = (uint32_t)start;
        });
    if (threadIdx.x == 0) {
        b.tile_start[ntiles] = (uint32_t)total;
        if (fits) atomicOr(b.status, kStatusFits);
    }
}

// Compact layout, second pass: bin every point again into the scanned layout.
// Every launch first clears the next binning's counters.
__global__ void __launch_bounds__(kGeoThreads) bin_scatter_kernel(GeoParams g, Binned b, int64_t n,
                                                                  int ntiles,
                                                                  const double *__restrict__ x,
                                                                  const double *__restrict__ y,
                                                                  const double *__restrict__ d,
                                                                  int64_t stride) {
    for (int i = blockIdx.x * kGeoThreads + threadIdx.x; i < ntiles; i += gridDim.x * kGeoThreads)
        b.next_cursor[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) b.next_status[0] = 0u;
    if (!(b.status[0] & kStatusCompact)) return;   // every slab held its tile
    const int64_t per = (int64_t)kGeoThreads * kBinPoints;
    const int64_t nblk = (n + per - 1) / per;
    for (int64_t i = blockIdx.x; i < nblk; i += gridDim.x)
        bin_block<false>(g, b, n, scattered_block(i, stride, nblk), x, y, d);
}

}  // namespace

// The stride of scattered_block for nblk blocks: coprime to nblk, near 0.618 nblk.
int64_t scatter_stride(int64_t nblk) {
    int64_t st = (int64_t)(0.6180339887498949 * (double)nblk);
    if (st < 1) st = 1;
    for (;; ++st) {
        int64_t a = st, c = nblk;
        while (c) {
            const int64_t t = a % c;
            a = c;
            c = t;
        }
        if (a == 1) return st;
    }
}

hipError_t launch_bin_reset(const Binned &b, int ntiles, hipStream_t s) {
    const int blocks = ((ntiles > kSplitSlots ? ntiles : kSplitSlots) + 255) / 256;
    hipLaunchKernelGGL(bin_reset_kernel, dim3(blocks), dim3(256), 0, s, b, ntiles);
    return hipGetLastError();
}

hipError_t launch_bin_fill(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                           const double *y, const double *d, hipStream_t s) {
    const int64_t per = (int64_t)kGeoThreads * kBinPoints;
    const int64_t blocks = (n + per - 1) / per;
    hipLaunchKernelGGL(bin_fill_kernel, dim3((unsigned)blocks), dim3(kGeoThreads), 0, s, g, b, n, x, y, d,
                       scatter_stride(blocks));
    return hipGetLastError();
}

hipError_t launch_bin_count(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                            const double *y, const double *d, hipStream_t s) {
    const int64_t per = (int64_t)kGeoThreads * kCountPoints;
    const int64_t blocks = (n + per - 1) / per;
    hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)blocks), dim3(kGeoThreads), 0, s, g, b, n, x, y, d);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Binned &b, int ntiles, int ntx, uint32_t slots, hipStream_t s) {
    if (ntx <= 0 || ntx > kMaxTileCols || (ntx & (ntx - 1)) || ntiles % ntx) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, b, ntiles, ntx, slots);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const GeoParams &g, const Binned &b, int64_t n, int ntiles, const double *x,
                              const double *y, const double *d, hipStream_t s) {
    const int64_t per = (int64_t)kGeoThreads * kBinPoints;
    const int64_t blocks = (n + per - 1) / per;
    const int grid = (int)(blocks < kFallbackBlocks ? blocks : kFallbackBlocks);
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(grid), dim3(kGeoThreads), 0, s, g, b, n, ntiles, x, y, d,
                       scatter_stride(blocks));
    return hipGetLastError();
}

}  // namespace asf
