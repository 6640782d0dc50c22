// Spreading on gfx950: the "interpolation" half of the non-uniform FFT the
// paper evaluates Eq. (9) with (Sec. 2).  Each binned point carries
// c_j = u1_j exp(i phi_j) and adds c_j psi(l_x - g_x) psi(l_y - g_y) to the w x w
// fine cells around its position g (periodic), where psi is the
// exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)).
//
// One workgroup owns one tile of the fine grid.  Its bin lists every point whose
// footprint touches the tile, so the workgroup accumulates whole footprints
// into an LDS tile padded by w-1 cells on each side (no clipping), then writes
// only its own cells -- every fine cell of a tile some record reaches is written
// exactly once with plain stores, no global atomics and no separate clear of the
// fine grid.  Where the plan asks for it, a tile no record reaches is not written at
// all: the binning flags it 0 and the column pass reads its cells as zeros
// (geometries whose frequencies cover part of the fine grid leave most tiles so).
//
// Kernel values.  psi at the w cells of a footprint is a polynomial in the
// point's cell offset f (es_poly.h, FP64 Chebyshev interpolants, within 1e-7 of
// psi at w = 7); psi is even, so the cells i and w-1-i share the even and odd
// parts of one polynomial: about w + 3 FMAs per pair of cells instead of an
// exp and a sqrt per cell.
//
// Accumulation is in fixed point with LDS integer atomics: on gfx950 an LDS
// float atomic add runs about one lane at a time, the integer ones at full LDS
// rate.  A term t is made an integer by y = fma(a, k, 1.5 * 2^23): for
// |t| < 2^22 the float y lies in [2^23, 2^24), where floats are the integers,
// so the FMA rounds the exact product to the nearest integer (ties to even:
// unbiased, which matters because a bias per term would add up coherently over
// ~1e9 terms at the lowest modes) and the bit pattern of y is
// 0x4B400000 + round(t).  One 64-bit integer add of a constant then removes the
// 0x4B400000 offsets.  Per tile, M = max(|Re c_j|, |Im c_j|) over its points
// bounds every term's parts.  A tile of at most 1023 records gives no cell more
// than 1023 terms; its terms are scaled to below 2^21 (rounding step 2^-21 M)
// and packed.  Larger tiles count the footprints starting in each cell: K = w^2
// times the most of them bounds the terms any cell receives; terms are scaled
// to below 2^22 (rounding step 2^-22 M), and
//   packed (K <= 511): no cell sum leaves int32 (511 (2^22 + 1/2) < 2^31, and
//            1023 (2^21 + 1/2) < 2^31), so one 64-bit word holds Re + 2^32 Im:
//            a single ds_add_u64 adds both parts of a term (the carry of the low
//            half into the high half is undone exactly at unpacking);
//   split:   denser tiles, and grids so small that the padded tile folds onto
//            itself, keep separate 64-bit sums of Re and Im, accumulated in two
//            sweeps over the same LDS array, with 42-bit terms (term42: the
//            rounding remainder of each term kept as a second 20-bit piece).
// One rounding step for every term of a tile costs a tile whose weight sits in a
// few records (a bright point among weak ones) more than the others: their
// rounding error is set by the bright record's amplitude, not by their own.
// Such tiles (nonzero parts averaging 4 or more octaves below the largest) take
// the split sums as well.  Every decision of a tile comes from maxima and integer
// counts, and integer addition is associative, so the spread is bitwise
// deterministic and independent of the order the binning left the records in.
//
// Crowded tiles.  A tile far above the mean load of a resident workgroup (the
// binning's scan decides, from the record counts) is cut into slices of
// consecutive records, each taken by its own workgroup.  The slices share one
// scale -- the largest |u1| among all the tile's records -- and the split sums,
// write their integer sums to a partial buffer, and the last slice to finish
// adds them (exactly) and writes the tile.
//
// Bank conflicts.  A wave's 64 lanes add the same footprint offset to 64
// different points, so lane l touches base_l + const; LDS serves a quarter wave
// at a time, conflict-free when the 16 bases are distinct modulo 16 cells.
// Random bases put about three lanes on the busiest residue, and in dense
// regions whole quarter waves can hit one cell, so the records of a tile are
// counting-sorted by that residue in LDS and dealt out column-wise: lane i of a
// quarter wave takes sorted entry i * ceil(n/16) + q, so a quarter wave draws
// one entry from each sixteenth of the sorted list -- distinct residues unless
// a residue class is larger than n/16.  Only tiles with a handful of records
// skip the sort and add from registers.  Measured on gfx950, ds_add_u64 runs at
// ~10 lanes/clk/CU conflict-free and ~6 with random addresses.
//
// The fine grid is stored in panels of `panel` adjacent columns: element
// (gx, gy) lives at ((gx / panel) * nfy + gy) * panel + gx % panel, so that the
// first FFT pass reads a panel of columns as one contiguous block.
#include "asf_internal.h"
#include "es_poly.h"

namespace asf {
namespace {

constexpr int kTileXMax = 64;
constexpr int kTileYMax = 32;
constexpr int kThreads = 512;
constexpr int kBatch = 2;                 // records per thread held in registers
constexpr int kChunk = 2 * kThreads;      // records sorted and dealt at a time
constexpr int kWavesPerSimd = 6;          // three 512-thread workgroups per CU (LDS allows three)

template <int W>
struct TileGeom {
    static constexpr int PAD = W - 1;
    // LDS row pitch (cells), = 2 mod 16: the write-out reads 16 lanes as 8 rows x 2
    // adjacent columns, which then fall in 16 distinct bank pairs
    static constexpr int PITCH = (kTileXMax + 2 * PAD - 2 + 15) / 16 * 16 + 2;
    static constexpr int ROWS = kTileYMax + 2 * PAD;
    static constexpr int CELLS = PITCH * ROWS;
};

// psi at the w footprint cells for offset f in [-1/2, 1/2]
template <int W>
__device__ inline void es_values(float f, float (&v)[W]) {
    constexpr int D = es_poly_degree(W);
    const float u = f * f;
#pragma unroll
    for (int i = 0; i < (W + 1) / 2; ++i) {
        float e = kEsPoly[W - 2][i][D & ~1];
#pragma unroll
        for (int k = (D & ~1) - 2; k >= 0; k -= 2) e = __builtin_fmaf(e, u, kEsPoly[W - 2][i][k]);
        if (2 * i == W - 1) {
            v[i] = e;
        } else {
            constexpr int DO = (D - 1) | 1;   // highest odd power
            float o = kEsPoly[W - 2][i][DO];
#pragma unroll
            for (int k = DO - 2; k >= 1; k -= 2) o = __builtin_fmaf(o, u, kEsPoly[W - 2][i][k]);
            v[i] = __builtin_fmaf(f, o, e);
            v[W - 1 - i] = __builtin_fmaf(-f, o, e);
        }
    }
}

constexpr float kMagic = 12582912.f;             // 1.5 * 2^23
constexpr unsigned kMagicBits = 0x4B400000u;      // bit pattern of kMagic
constexpr unsigned long long kMagic1 = kMagicBits;
constexpr unsigned long long kMagic2 = ((unsigned long long)kMagicBits << 32) | kMagicBits;

// round(a k) as a 64-bit two's-complement integer, for |a k| < 2^22
__device__ inline unsigned long long term1(float a, float k) {
    return (unsigned long long)__float_as_uint(__builtin_fmaf(a, k, kMagic)) - kMagic1;
}

// round(re) + 2^32 round(im) modulo 2^64, for |re|, |im| < 2^22
__device__ inline unsigned long long term(float ar, float ai, float k) {
    const float yr = __builtin_fmaf(ar, k, kMagic);
    const float yi = __builtin_fmaf(ai, k, kMagic);
    return (((unsigned long long)__float_as_uint(yi) << 32) | __float_as_uint(yr)) - kMagic2;
}

// round(a k 2^20) as a 64-bit integer to within one unit, for |a k| < 2^22 (the
// split sums of crowded or high-dynamic-range tiles): round(a k) from the FMA above,
// then the remainder a k - round(a k) (|.| <= 1/2, formed exactly by a second FMA and
// rounded once to FP32) scaled by 2^20 and rounded the same way.  Both roundings are
// to nearest even, so the terms stay unbiased.
__device__ inline unsigned long long term42(float a, float k) {
    const float y = __builtin_fmaf(a, k, kMagic);
    const float h = y - kMagic;
    const float r = __builtin_fmaf(a, k, -h);
    const float z = __builtin_fmaf(r, 0x1p20f, kMagic);
    const long long hi = (int)(__float_as_uint(y) - kMagicBits);
    const long long lo = (int)(__float_as_uint(z) - kMagicBits);
    return (unsigned long long)(hi * (1ll << 20) + lo);
}

__device__ inline void unpack2(unsigned long long v, int &re, int &im) {
    re = (int)(unsigned)(v & 0xffffffffull);
    im = (int)(unsigned)((v - (unsigned long long)(long long)re) >> 32);
}

// padded start position of a point in this tile, or false if it does not touch it
__device__ inline bool local_start(uint32_t cell, int x0, int y0, int pad, int hix, int hiy,
                                   int nfx, int nfy, int &px, int &py) {
    px = (int)(cell & 0xffffu) - x0 + pad;
    if (px < 0) px += nfx;
    else if (px > hix) px -= nfx;
    py = (int)(cell >> 16) - y0 + pad;
    if (py < 0) py += nfy;
    else if (py > hiy) py -= nfy;
    return px >= 0 && px <= hix && py >= 0 && py <= hiy;
}

// the records of one batch: slot base + k * nt for k < kBatch.  Until the u1
// gather pc holds exp(i phi); after it, c = u1 exp(i phi) (unscaled).
struct Batch {
    uint32_t j[kBatch], cell[kBatch];
    float2 fr[kBatch], pc[kBatch];
};

// binned record fields (the u1 gather is separate so that it can be issued later,
// once the indices have arrived)
// Every load is issued unconditionally (slots past s1 are clamped to s1 - 1, a
// record of the same tile, and then discarded), so that all of a thread's loads
// are in flight together instead of each waiting behind a branch.  s0 < s1.
__device__ inline void load_records(Batch &r, const Binned &b, uint32_t base, uint32_t s1, int nt) {
    uint2 kv[kBatch];
    float2 fr[kBatch], ph[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        const uint32_t s = min(base + k * nt, s1 - 1u);
        const float2 *rv = reinterpret_cast<const float2 *>(b.rec + s);
        kv[k] = b.key[s];
        fr[k] = rv[0];
        ph[k] = rv[1];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        const bool in = base + k * nt < s1;
        r.j[k] = in ? kv[k].y : 0xffffffffu;
        r.cell[k] = kv[k].x;
        r.fr[k] = in ? fr[k] : make_float2(0.f, 0.f);
        r.pc[k] = in ? ph[k] : make_float2(0.f, 0.f);
    }
}

// (indices past the point count, which only discarded slots carry, are clamped)
__device__ inline void gather_u(Batch &r, const float2 *__restrict__ u1, int64_t n) {
    float2 u[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) u[k] = u1[min((int64_t)r.j[k], n - 1)];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        if (r.j[k] >= n) u[k] = make_float2(0.f, 0.f);
        const float2 ph = r.pc[k];
        r.pc[k] = make_float2(u[k].x * ph.x - u[k].y * ph.y, u[k].x * ph.y + u[k].y * ph.x);
    }
}

template <int W, int PITCH>
__device__ inline void accumulate(unsigned long long *row, float4 d, bool packed) {
    float kx[W], ky[W];
    es_values<W>(d.z, kx);
    es_values<W>(d.w, ky);
#pragma unroll
    for (int jy = 0; jy < W; ++jy) {
        const float ar = d.x * ky[jy], ai = d.y * ky[jy];
        if (packed) {
#pragma unroll
            for (int i = 0; i < W; ++i) atomicAdd(row + jy * PITCH + i, term(ar, ai, kx[i]));
        } else {
#pragma unroll
            for (int i = 0; i < W; ++i) atomicAdd(row + jy * PITCH + i, term42(ar, kx[i]));
        }
    }
}

// Tiles with more records than this deal them out by start residue (see the
// file comment); the few lighter ones add their footprints straight from
// registers, where the sort would cost more than the conflicts it removes.
// (Measured on the 2048^2 cap: dealing every tile with more than 64 records
// takes the spread from 0.159 to 0.144 ms; a threshold of 1024 left most of its
// tiles conflicted.)
constexpr uint32_t kDealRecords = 64;
// Tiles of at most this many records skip the start histogram and pack their
// cells with terms below 2^21: no cell sum can leave int32.
constexpr uint32_t kFewRecords = 1023;

// The tile's own cells are read back and written out in panel order: thread tid
// handles cells tid + k nt; with nt a multiple of panel * tile_y it keeps its row
// ly and column offset lx, and successive k step col_step = nt / tile_y columns
// (col_step nfy elements in the fine grid's panel layout).
struct TileCells {
    int lx, ly, col_step;
    size_t grid, grid_step;
};

__device__ inline TileCells tile_cells(const SpreadParams &p, int x0, int y0, int nt) {
    const int tid = threadIdx.x;
    const int C = 1 << p.log_panel;
    const int c = tid & (C - 1);
    const int rest = tid >> p.log_panel;
    TileCells m;
    m.ly = rest & ((1 << p.log_tile_y) - 1);
    m.lx = ((rest >> p.log_tile_y) << p.log_panel) + c;
    m.col_step = nt >> p.log_tile_y;
    m.grid = (((size_t)((x0 + m.lx) >> p.log_panel) * p.nfy + y0 + m.ly) << p.log_panel) + c;
    m.grid_step = (size_t)m.col_step * p.nfy;
    return m;
}

// The tile's own cells as FP32 into the fine grid.
template <int W, int PITCH>
__device__ inline void write_tile(const unsigned long long *acc, float2 *__restrict__ fine,
                                  const SpreadParams &p, int x0, int y0, int ncell, int nt, bool packed,
                                  int sweep, float unscale) {
    constexpr int PAD = W - 1;
    const TileCells m = tile_cells(p, x0, y0, nt);
    const unsigned long long *src = acc + (m.ly + PAD) * PITCH + m.lx + PAD;
    float2 *dst = fine + m.grid;
    for (int k = 0; k < ncell / nt; ++k) {
        const unsigned long long v = src[k * m.col_step];
        float2 *d = dst + k * m.grid_step;
        if (packed) {
            int sr, si;
            unpack2(v, sr, si);
            *d = make_float2((float)sr * unscale, (float)si * unscale);
        } else {
            // split tiles: sweep 0 writes the real part, sweep 1 the imaginary part
            reinterpret_cast<float *>(d)[sweep] = (float)(long long)v * unscale;
        }
    }
}

// A slice of a cut tile: its integer sums (one sweep's part) in write-out order.
template <int W, int PITCH>
__device__ inline void write_partial(const unsigned long long *acc, unsigned long long *__restrict__ part,
                                     const SpreadParams &p, int ncell, int nt) {
    constexpr int PAD = W - 1;
    const TileCells m = tile_cells(p, 0, 0, nt);
    const unsigned long long *src = acc + (m.ly + PAD) * PITCH + m.lx + PAD;
    for (int k = 0; k < ncell / nt; ++k) part[k * nt + threadIdx.x] = src[k * m.col_step];
}

// The last slice of a cut tile to finish adds the slices' integer sums (exact: the
// result does not depend on how the records were dealt to slices, nor on which
// slice ends last) and writes the tile.  part: [slices][2][ncell], Re then Im.
// The tile's cells are kCombineCells per thread (ncell = 2048 = 4 nt on the grids
// that cut tiles); each step loads kCombineSlices slices' sums of all of them, 32
// loads in flight.
constexpr int kCombineCells = 4;
constexpr int kCombineSlices = 4;
static_assert(kTileXMax * kTileYMax == kCombineCells * kThreads, "cut tiles are full 64 x 32 tiles");

__device__ inline void combine_tile(const unsigned long long *part, uint32_t nsl, float2 *__restrict__ fine,
                                    const SpreadParams &p, int x0, int y0, int ncell, int nt, float unscale) {
    const TileCells m = tile_cells(p, x0, y0, nt);
    unsigned long long re[kCombineCells] = {}, im[kCombineCells] = {};
    const unsigned long long *src = part + threadIdx.x;
    for (uint32_t q = 0; q < nsl; q += kCombineSlices) {
        unsigned long long v[kCombineSlices][2][kCombineCells];
#pragma unroll
        for (int h = 0; h < kCombineSlices; ++h) {
            const uint32_t qh = min(q + h, nsl - 1u);   // past the last slice: reloaded, added as zero
#pragma unroll
            for (int k = 0; k < kCombineCells; ++k) {
                v[h][0][k] = src[(size_t)(2 * qh) * ncell + k * nt];
                v[h][1][k] = src[(size_t)(2 * qh + 1) * ncell + k * nt];
            }
        }
#pragma unroll
        for (int h = 0; h < kCombineSlices; ++h) {
            const unsigned long long keep = q + h < nsl ? ~0ull : 0ull;
#pragma unroll
            for (int k = 0; k < kCombineCells; ++k) {
                re[k] += v[h][0][k] & keep;
                im[k] += v[h][1][k] & keep;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kCombineCells; ++k)
        fine[m.grid + k * m.grid_step] = make_float2((float)(long long)re[k] * unscale, (float)(long long)im[k] * unscale);
}

// Wave-wide reductions by lane permutations on the vector ALU (DPP): within each
// row of 16 lanes, exchanges with lane ^ 1 and lane ^ 2, then the half-row and row
// mirrors leave every lane with its row's result; four lane reads combine the
// rows.  A few cycles per step, where shuffles routed through the LDS crossbar
// take a round trip each.
__device__ inline unsigned dpp_row_max(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row half mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
    return v;
}

__device__ inline unsigned dpp_row_sum(unsigned v) {
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
    return v;
}

// inclusive prefix sum within each row of 16 lanes (row shifts by 1, 2, 4, 8;
// lanes shifted in from outside the row read 0)
__device__ inline unsigned dpp_row_prefix(unsigned v) {
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    return v;
}

// (the whole wave must be active; the result is uniform)
__device__ inline unsigned wave_max(unsigned v) {
    v = dpp_row_max(v);
    return max(max((unsigned)__builtin_amdgcn_readlane((int)v, 0), (unsigned)__builtin_amdgcn_readlane((int)v, 16)),
               max((unsigned)__builtin_amdgcn_readlane((int)v, 32), (unsigned)__builtin_amdgcn_readlane((int)v, 48)));
}

__device__ inline unsigned wave_sum(unsigned v) {
    v = dpp_row_sum(v);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 0) + (unsigned)__builtin_amdgcn_readlane((int)v, 16) +
           (unsigned)__builtin_amdgcn_readlane((int)v, 32) + (unsigned)__builtin_amdgcn_readlane((int)v, 48);
}

// A tile whose weight sits in a few of its records: the exponents of its nonzero
// parts (max(|Re c|, |Im c|) per record) average 4 or more below the largest one,
// E.  The packed sums round every term to 2^-21 M (or 2^-22 M), M the largest part,
// which costs the other records a relative error set by M rather than by their own
// size: about 1.5e-6 for a tile of random phases and amplitudes, 2e-5 for one
// bright point among 500 points 1e4 times weaker.  Such tiles take the split sums
// with 42-bit terms.  (Zero records add exact zeros and do not count.)  The
// statistic is a sum of integer exponents, so this decision, like the tile's
// others (maxima and counts), does not depend on the order the binning left the
// records in.
__device__ inline bool high_dynamic_range(unsigned ebig, unsigned long long nnz, unsigned long long esum) {
    return nnz > 0ull && ebig * nnz - esum >= 4ull * nnz;
}

// Exponent bound of the terms of a split tile: each record adds at most one term
// to a cell, so a cell sum of nrec terms below 2^(emax + 20) (term42) stays below
// 2^62 when emax + 20 + log2(nrec) <= 62.
__device__ inline int split_emax(uint32_t nrec) {
    int lg = 0;
    while (lg < 32 && (1u << lg) < nrec) ++lg;
    return min(22, 42 - lg);
}

template <int W>
__global__ void __launch_bounds__(kThreads, kWavesPerSimd) spread_kernel(SpreadParams p, Binned b,
                                                          const float2 *__restrict__ u1,
                                                          float2 *__restrict__ fine) {
    using G = TileGeom<W>;
    constexpr int PAD = G::PAD;
    constexpr int PITCH = G::PITCH;
    constexpr int SWMAX = (kTileXMax + PAD) * (kTileYMax + PAD);
    constexpr int SDAT = (kChunk + 16) > (SWMAX + 3) / 4 ? (kChunk + 16) : (SWMAX + 3) / 4;
    __shared__ __align__(16) unsigned long long acc[G::CELLS];
    __shared__ __align__(16) float4 sdat[SDAT];          // dealt records (Re c, Im c, fx, fy)
    __shared__ int sbase[kChunk + 16];                   // their padded start cell
    __shared__ unsigned rcount[16];                      // records per start residue
    __shared__ unsigned sbig, smost;                     // block maxima
    __shared__ unsigned long long snnz, sesum;           // nonzero records, sum of their exponents
    int *starts = reinterpret_cast<int *>(sdat);         // footprint-start histogram (phase A)

    // this workgroup's tile, and its slice of the records if the tile is cut
    int t;
    uint32_t slice, nsl, slot, s0, s1;
    if (!tile_work(b, p.ntx * p.nty, t, slice, nsl, slot, s0, s1)) return;
    const int tsx = 1 << p.log_tile_x, tsy = 1 << p.log_tile_y;
    const int ext_x = tsx + 2 * PAD, ext_y = tsy + 2 * PAD;   // padded tile extent
    const int swx = tsx + PAD, swy = tsy + PAD;               // start positions per axis
    const int hix = swx - 1, hiy = swy - 1;
    const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const bool fold_x = p.nfx < ext_x, fold_y = p.nfy < ext_y;
    const int ncell = tsx * tsy;
    const uint32_t per_batch = (uint32_t)(kBatch * nt);
    const int ty = t >> p.log_ntx, tx = t & ((1 << p.log_ntx) - 1);
    const int x0 = tx << p.log_tile_x, y0 = ty << p.log_tile_y;
    const uint32_t nrec = s1 - s0;
    const bool reload = nrec > per_batch;
    const bool deal = nrec > kDealRecords;
    // The slices of a cut tile all take the split sums with 42-bit terms at one
    // scale, set by the largest |u1| among all the tile's records (|exp(i phi)| = 1
    // bounds |Re c| and |Im c| by it): every term is then the same integer whichever
    // slice adds it, and the slices' sums add up exactly to the whole tile's.
    const bool cut = nsl > 1;
    // a tile no record reaches (flagged 0 by the binning) may be left unwritten: the
    // column pass then reads its cells as zeros
    if (p.skip_dead && nrec == 0) return;
    // a tile of few records needs no start histogram: no cell receives more than
    // nrec terms (unless the grid folds the padded tile onto itself: split sums)
    const bool few = nrec <= kFewRecords && !fold_x && !fold_y && !cut;
    const bool count_starts = !few && !cut;
    {
        uint4 *a4 = reinterpret_cast<uint4 *>(acc);
        for (int i = tid; i < G::CELLS / 2; i += nt) a4[i] = make_uint4(0u, 0u, 0u, 0u);
        if (count_starts)
            for (int i = tid; i < swx * swy; i += nt) starts[i] = 0;
        if (tid < 16) rcount[tid] = 0u;
        if (tid == 0) {
            sbig = smost = 0u;
            snnz = sesum = 0ull;
        }
    }
    Batch r;
    int rb[kBatch];   // padded start cell of each record, -1 if it does not touch the tile
    __syncthreads();

    // phase A: largest |Re c| or |Im c| (and, for larger tiles, the count of
    // footprint starts per position).  A tile of at most kBatch * nt records
    // keeps them in registers for phase B; larger tiles reload them there.
    float big = 0.f;
    unsigned nnz = 0u, esum = 0u;   // this thread's nonzero parts and the sum of their exponents
    for (uint32_t base = s0; base < s1; base += per_batch) {
        load_records(r, b, base + tid, s1, nt);
        gather_u(r, u1, p.n);
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            int px, py;
            rb[k] = -1;
            if (r.j[k] < p.n && local_start(r.cell[k], x0, y0, PAD, hix, hiy, p.nfx, p.nfy, px, py)) {
                rb[k] = py * PITCH + px;
                const float part = fmaxf(fabsf(r.pc[k].x), fabsf(r.pc[k].y));
                big = fmaxf(big, part);
                // branch-free: a zero part adds exponent 0 and no count
                nnz += part > 0.f ? 1u : 0u;
                esum += __float_as_uint(part) >> 23;
                if (count_starts) atomicAdd(&starts[py * swx + px], 1);
            }
        }
    }
    uint32_t tile_records = nrec;
    if (cut) {
        // the scale of all the tile's slices: the largest |u1| over all its records,
        // eight records per thread in flight
        uint32_t a0, a1;
        tile_slots(b, t, a0, a1);
        tile_records = a1 - a0;
        big = 0.f;
        constexpr int kScan = 8;
        for (uint32_t i = a0 + tid; i < a1; i += kScan * nt) {
            uint32_t j[kScan];
            float2 u[kScan];
#pragma unroll
            for (int q = 0; q < kScan; ++q) j[q] = b.key[min(i + q * nt, a1 - 1u)].y;
#pragma unroll
            for (int q = 0; q < kScan; ++q) u[q] = u1[min((int64_t)j[q], p.n - 1)];
#pragma unroll
            for (int q = 0; q < kScan; ++q)
                if (i + q * nt < a1 && j[q] < p.n) big = fmaxf(big, sqrtf(u[q].x * u[q].x + u[q].y * u[q].y));
        }
    }
    // block maximum (non-negative floats order like their bit patterns) and the
    // exponent statistics: wave sums in 32 bits (a wave holds an eighth of the
    // tile's records; tiles of 2^24 or more records skip the statistic), 64-bit
    // sums across the block
    const unsigned wbig = wave_max(__float_as_uint(big));
    const unsigned wnnz = wave_sum(nnz), wesum = wave_sum(esum);
    if (lane == 0) {
        atomicMax(&sbig, wbig);
        if (!cut && wnnz) {
            atomicAdd(&snnz, (unsigned long long)wnnz);
            atomicAdd(&sesum, (unsigned long long)wesum);
        }
    }
    __syncthreads();               // sbig, snnz, sesum and starts[] complete
    big = __uint_as_float(sbig);
    bool packed;
    int emax;                      // terms are bounded by 2^emax
    if (cut) {
        packed = false;
        emax = split_emax(tile_records);
    } else if (few) {
        packed = true;             // kFewRecords (2^21 + 1/2) < 2^31
        emax = 21;
    } else {
        unsigned most = 0u;        // most footprint starts in one cell
        for (int i = tid; i < swx * swy; i += nt) most = max(most, (unsigned)starts[i]);
        most = wave_max(most);
        if (lane == 0) atomicMax(&smost, most);
        __syncthreads();
        // 511 (2^22 + 1/2) < 2^31; grids folding the tile onto itself sum several cells
        packed = smost * (unsigned)(W * W) <= 511u && !fold_x && !fold_y;
        emax = 22;
    }
    // a few records dominating the tile: the others would be rounded on the dominant
    // ones' grid, so the tile takes the split sums with 42-bit terms
    if (!cut) {
        if (nrec >= (1u << 24) || high_dynamic_range(sbig >> 23, snnz, sesum)) packed = false;
        if (!packed) emax = split_emax(nrec);
    }
    int e = 0;
    if (big > 0.f) {
        int em;
        frexpf(big * (1.f + 0x1p-18f), &em);   // margin for rounding in c and psi
        e = emax - em;
    }
    e = max(-120, min(e, 120));
    const float scale = ldexpf(1.f, e);
    // split sums carry 20 more fractional bits (term42)
    const float unscale = ldexpf(1.f, packed ? -e : -e - 20);

    // phase B: accumulate every footprint (split tiles: two sweeps, Re then Im)
    const int sweeps = packed ? 1 : 2;
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (uint32_t bb = s0; bb < s1; bb += per_batch) {
            if (reload) {
                load_records(r, b, bb + tid, s1, nt);
                gather_u(r, u1, p.n);
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    int px, py;
                    rb[k] = (r.j[k] < p.n && local_start(r.cell[k], x0, y0, PAD, hix, hiy, p.nfx, p.nfy, px, py))
                                ? py * PITCH + px : -1;
                }
            }
            if (!deal) {
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    if (rb[k] < 0) continue;
                    const float cr = r.pc[k].x * scale, ci = r.pc[k].y * scale;
                    // split sweep 0 adds Re, sweep 1 adds Im, each alone
                    const float c0 = packed ? cr : (sweep == 0 ? cr : ci);
                    accumulate<W, PITCH>(acc + rb[k], make_float4(c0, ci, r.fr[k].x, r.fr[k].y), packed);
                }
                continue;
            }
#pragma unroll
            for (int h = 0; h < kBatch / 2; ++h) {
                if (bb + (uint32_t)(h * 2 * nt) >= s1) break;   // uniform over the block
                // sort this chunk's records by start residue: rank within class
                float4 rec[2];
                int rres[2];
                unsigned rrank[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int k = 2 * h + q;
                    const float cr = r.pc[k].x * scale, ci = r.pc[k].y * scale;
                    const float c0 = packed ? cr : (sweep == 0 ? cr : ci);
                    rec[q] = make_float4(c0, ci, r.fr[k].x, r.fr[k].y);
                    rres[q] = rb[k] & 15;
                    rrank[q] = rb[k] >= 0 ? atomicAdd(&rcount[rres[q]], 1u) : 0u;
                }
                __syncthreads();   // residue counts complete
                // exclusive prefix of the 16 counts, held by lanes 0..15 of every wave
                const unsigned cnt = lane < 16 ? rcount[lane] : 0u;
                const unsigned inc = dpp_row_prefix(cnt);
                const unsigned total = (unsigned)__builtin_amdgcn_readlane((int)inc, 15);
                const unsigned excl = inc - cnt;
                const unsigned n16 = (total + 15u) >> 4;
                const float inv16 = n16 ? 1.f / (float)n16 : 0.f;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    // sorted position, then the column-wise deal: position srt goes
                    // to slot (srt mod n16) * 16 + srt / n16 (the quotient is exact:
                    // the float estimate of (srt + 1/2) / n16 is >= 1/128 from an
                    // integer)
                    const unsigned srt = rrank[q] + __shfl(excl, rres[q]);
                    if (rb[2 * h + q] < 0) continue;
                    const unsigned quo = (unsigned)(((float)srt + 0.5f) * inv16);
                    const unsigned slot = (srt - quo * n16) * 16u + quo;
                    sdat[slot] = rec[q];
                    sbase[slot] = rb[2 * h + q];
                }
                __syncthreads();   // records dealt; counts read by everyone
                if (tid < 16) rcount[tid] = 0u;
#pragma unroll 1
                for (int q = 0; q < 2; ++q) {
                    const unsigned s = (unsigned)(tid + q * nt);
                    if ((s >> 4) >= n16 || (s & 15u) * n16 + (s >> 4) >= total) continue;
                    accumulate<W, PITCH>(acc + sbase[s], sdat[s], packed);
                }
                __syncthreads();   // staging reused by the next chunk
            }
        }
        __syncthreads();

        if (cut) {
            // slices are only made on grids that do not fold
            write_partial<W, PITCH>(acc, b.partial + (size_t)(2 * (slot + slice) + sweep) * ncell, p, ncell, nt);
        } else if (!fold_x && !fold_y) {
            write_tile<W, PITCH>(acc, fine, p, x0, y0, ncell, nt, packed, sweep, unscale);
        } else {
            // grids narrower than the padded tile: fold the wrapped halo back in
            const int C = 1 << p.log_panel;
            for (int i = tid; i < ncell; i += nt) {
                const int c = i & (C - 1);
                const int rest = i >> p.log_panel;
                const int ly = rest & (tsy - 1);
                const int lx = ((rest >> p.log_tile_y) << p.log_panel) + c;
                unsigned long long v = 0ull;
                for (int oy = ly + PAD - 2 * p.nfy; oy < ext_y; oy += p.nfy) {
                    if (oy < 0 || (!fold_y && oy != ly + PAD)) continue;
                    for (int ox = lx + PAD - 2 * p.nfx; ox < ext_x; ox += p.nfx) {
                        if (ox < 0 || (!fold_x && ox != lx + PAD)) continue;
                        v += acc[oy * PITCH + ox];
                    }
                }
                float2 *dst = fine + ((((size_t)((x0 + lx) >> p.log_panel) * p.nfy + y0 + ly) << p.log_panel) + c);
                if (packed) {
                    int sr, si;
                    unpack2(v, sr, si);
                    *dst = make_float2((float)sr * unscale, (float)si * unscale);
                } else {
                    reinterpret_cast<float *>(dst)[sweep] = (float)(long long)v * unscale;
                }
            }
        }
        if (sweep + 1 < sweeps) {
            __syncthreads();
            uint4 *a4 = reinterpret_cast<uint4 *>(acc);
            for (int i = tid; i < G::CELLS / 2; i += nt) a4[i] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
        }
    }
    if (cut) {
        // partial sums stored: make them visible device-wide, then count the slice in;
        // the last of the tile's slices (whichever it is) reads all partials back
        __shared__ unsigned slast;
        __threadfence();
        __syncthreads();
        if (tid == 0) slast = atomicAdd(&b.combine[slot], 1u) == nsl - 1;
        __syncthreads();
        if (slast) {
            __threadfence();
            combine_tile(b.partial + (size_t)2 * slot * ncell, nsl, fine, p, x0, y0, ncell, nt, unscale);
            if (tid == 0) b.combine[slot] = 0u;   // ready for the next launch
        }
    }
}

template <int W>
hipError_t launch_w(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                    hipStream_t s) {
    const int groups = p.ntx * p.nty + (p.split ? kSplitSlots : 0);
    hipLaunchKernelGGL(spread_kernel<W>, dim3(groups), dim3(kThreads), 0, s, p, b, u1, fine);
    return hipGetLastError();
}

// Interpolation, the adjoint of spreading (the type-2 direction): every point
// gathers its w x w footprint of the fine grid with the same kernel weights,
//   g_j = conj(exp(i phi_j)) sum_l psi(l_x - g_x) psi(l_y - g_y) F[l],
// the conjugate pre-phase being the adjoint of the pre-phase multiply.  One
// workgroup per tile copies into LDS the cells the footprints of the tile's own
// points reach (the tile plus w-1 cells right and below, periodic).  A point is
// handled in the tile that holds its first footprint cell and skipped in the
// other bins that list it, so each point is written once, with a plain store:
// no atomics, and FP32 sums in registers.  Only footprint cells enter the sums:
// every one lies in a tile whose bin lists the point, so cells of tiles no record
// reaches (which the column pass may leave unwritten) are copied but never used.
constexpr int kInterpThreads = 256;

template <int W>
__global__ void __launch_bounds__(kInterpThreads) interp_kernel(SpreadParams p, Binned b,
                                                                const float2 *__restrict__ fine,
                                                                float2 *__restrict__ g1) {
    constexpr int RP = kTileXMax + W - 1;   // LDS row pitch (cells)
    __shared__ float2 reg[(kTileYMax + W - 1) * RP];
    // this workgroup's tile, and its slice of the records if the tile is cut (no
    // combining: every point is written by the one workgroup that holds its record)
    int t;
    uint32_t slice, nsl, slot, s0, s1;
    if (!tile_work(b, p.ntx * p.nty, t, slice, nsl, slot, s0, s1)) return;
    if (s0 == s1) return;   // no point to gather for: the region is not needed
    const int tsx = 1 << p.log_tile_x, tsy = 1 << p.log_tile_y;
    const int rx = tsx + W - 1, ry = tsy + W - 1;
    const int ty = t >> p.log_ntx, tx = t & ((1 << p.log_ntx) - 1);
    const int x0 = tx << p.log_tile_x, y0 = ty << p.log_tile_y;
    const int nt = blockDim.x, tid = threadIdx.x;
    // copy the region in the fine grid's panel order (C adjacent columns per row,
    // rows of a panel contiguous), so consecutive lanes read consecutive elements
    const int C = 1 << p.log_panel;
    const int rxp = (rx + C - 1) & ~(C - 1);
    const float inv_ry = 1.f / (float)ry;
    // kRegionLoads elements per thread in flight before their LDS writes
    constexpr int kRegionLoads = 6;
    for (int i0 = tid; i0 < rxp * ry; i0 += kRegionLoads * nt) {
        float2 v[kRegionLoads];
        int at[kRegionLoads];
#pragma unroll
        for (int q = 0; q < kRegionLoads; ++q) {
            const int i = i0 + q * nt;
            const int c = i & (C - 1);
            const int rest = i >> p.log_panel;
            const int qx = (int)(((float)rest + 0.5f) * inv_ry);   // rest / ry, exact for rest < 2^20
            const int yy = rest - qx * ry;
            const int xx = qx * C + c;
            at[q] = (i < rxp * ry && xx < rx) ? yy * RP + xx : -1;
            int gx = x0 + xx, gy = y0 + yy;
            if (gx >= p.nfx) gx -= p.nfx;
            if (gy >= p.nfy) gy -= p.nfy;
            v[q] = at[q] >= 0 ? fine[(((size_t)(gx >> p.log_panel) * p.nfy + gy) << p.log_panel) + (gx & (C - 1))]
                              : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < kRegionLoads; ++q)
            if (at[q] >= 0) reg[at[q]] = v[q];
    }
    __syncthreads();
    // two records per thread and iteration: their key and record loads all go out
    // together (slots past s1 clamped to s1 - 1 and discarded)
    for (uint32_t sb = s0 + tid; sb < s1; sb += 2 * nt) {
        uint2 kv[2];   // (cell, point index)
        float4 rv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t s = min(sb + q * nt, s1 - 1u);
            kv[q] = b.key[s];
            rv[q] = b.rec[s];
        }
        bool home[2];
        int px[2], py[2];
        uint32_t j[2];
        float2 fr[2], ph[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            px[q] = (int)(kv[q].x & 0xffffu) - x0;
            py[q] = (int)(kv[q].x >> 16) - y0;
            // a point is handled in its home tile only (and past s1 nowhere)
            home[q] = sb + q * nt < s1 && px[q] >= 0 && px[q] < tsx && py[q] >= 0 && py[q] < tsy;
            j[q] = home[q] ? kv[q].y : 0u;
            fr[q] = make_float2(rv[q].x, rv[q].y);
            ph[q] = make_float2(rv[q].z, rv[q].w);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (!home[q]) continue;
            float kx[W], ky[W];
            es_values<W>(fr[q].x, kx);
            es_values<W>(fr[q].y, ky);
            const float2 *row = reg + py[q] * RP + px[q];
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int jy = 0; jy < W; ++jy) {
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const float2 v = row[jy * RP + i];
                    sr = __builtin_fmaf(kx[i], v.x, sr);
                    si = __builtin_fmaf(kx[i], v.y, si);
                }
                ar = __builtin_fmaf(ky[jy], sr, ar);
                ai = __builtin_fmaf(ky[jy], si, ai);
            }
            // times conj(exp(i phi))
            g1[j[q]] = make_float2(ar * ph[q].x + ai * ph[q].y, ai * ph[q].x - ar * ph[q].y);
        }
    }
}

template <int W>
hipError_t launch_interp_w(const SpreadParams &p, const Binned &b, const float2 *fine, float2 *g1,
                           hipStream_t s) {
    const int groups = p.ntx * p.nty + (p.split ? kSplitSlots : 0);
    hipLaunchKernelGGL(interp_kernel<W>, dim3(groups), dim3(kInterpThreads), 0, s, p, b, fine, g1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_spread(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                         hipStream_t s) {
    if ((1 << p.log_tile_x) > kTileXMax || (1 << p.log_tile_y) > kTileYMax) return hipErrorInvalidValue;
    if ((1 << p.log_tile_x) % 16 != 0) return hipErrorInvalidValue;   // start residues need 16 | tile_x
    switch (p.w) {
        case 2: return launch_w<2>(p, b, u1, fine, s);
        case 3: return launch_w<3>(p, b, u1, fine, s);
        case 4: return launch_w<4>(p, b, u1, fine, s);
        case 5: return launch_w<5>(p, b, u1, fine, s);
        case 6: return launch_w<6>(p, b, u1, fine, s);
        case 7: return launch_w<7>(p, b, u1, fine, s);
        case 8: return launch_w<8>(p, b, u1, fine, s);
        case 9: return launch_w<9>(p, b, u1, fine, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp(const SpreadParams &p, const Binned &b, const float2 *fine, float2 *g1,
                         hipStream_t s) {
    if ((1 << p.log_tile_x) > kTileXMax || (1 << p.log_tile_y) > kTileYMax) return hipErrorInvalidValue;
    switch (p.w) {
        case 2: return launch_interp_w<2>(p, b, fine, g1, s);
        case 3: return launch_interp_w<3>(p, b, fine, g1, s);
        case 4: return launch_interp_w<4>(p, b, fine, g1, s);
        case 5: return launch_interp_w<5>(p, b, fine, g1, s);
        case 6: return launch_interp_w<6>(p, b, fine, g1, s);
        case 7: return launch_interp_w<7>(p, b, fine, g1, s);
        case 8: return launch_interp_w<8>(p, b, fine, g1, s);
        case 9: return launch_interp_w<9>(p, b, fine, g1, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace asf
