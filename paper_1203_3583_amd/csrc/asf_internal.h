// Internal declarations shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asf.h"

namespace asf {

// Binned point list: one slot per (point, fine-grid tile its footprint touches).
// Two layouts share the slot arrays.  Slab (the normal case): tile t owns the
// slots [slab[t].x, slab[t].x + slab[t].y), and cursor[t] counts its records
// (also past the slab's end).  The first slabs are uniform (4 n / ntiles slots
// each); a binning that needed the compact layout sizes new ones from its tile
// counts for the next binning.  Compact (after a slab overflowed): the tiles'
// records are packed in tile order, tile t in [tile_start[t], tile_start[t + 1]).
// Status bit kStatusCompact names the layout in use.
struct Binned {
    uint32_t *status;      // [1] kStatus* bits
    uint32_t *tile_start;  // [ntiles + 1] compact layout: exclusive scan of slot counts per tile
    uint32_t *cursor;      // [ntiles] slot counts; compact layout: then insertion cursors
    uint2 *slab;           // [ntiles] first slot and slot count of each tile's slab
    // a record in two words, each read or written by one instruction:
    uint2 *key;            // [slot_cap] (first footprint cell l0x | l0y << 16,
                           //             index j of the point in the caller's order)
    float4 *rec;           // [slot_cap] (gx - l0x - (w-1)/2, gy - l0y - (w-1)/2), each in
                           //            (-1/2, 1/2], then exp(i phi_j), the pre-phase of Eq. (8)
    uint32_t slot_cap;     // slots in the arrays above (4 n_src)
    // the other copy of status and cursor, which the next binning uses: the last
    // binning pass clears it, so that a binning needs no clearing launch of its own
    uint32_t *next_status;
    uint32_t *next_cursor;
};

constexpr uint32_t kStatusDomain = 1u;    // some point has r0 <= 0 or a non-finite coordinate
constexpr uint32_t kStatusOverflow = 2u;  // compact layout ran out of slots (internal error)
constexpr uint32_t kStatusCompact = 4u;   // the compact layout is in use
constexpr uint32_t kStatusFits = 8u;      // compact layout, and new slabs sized from its counts fit

// Slots [s0, s1) of tile t in whichever layout the last binning left.
__device__ inline void tile_slots(const Binned &b, int t, uint32_t &s0, uint32_t &s1) {
    if (b.status[0] & kStatusCompact) {
        s0 = b.tile_start[t];
        s1 = b.tile_start[t + 1];
    } else {
        const uint2 sl = b.slab[t];
        s0 = sl.x;
        s1 = s0 + min(b.cursor[t], sl.y);
    }
}

// Scalars the geometry kernels need (all FP64 where the paper's phases live).
struct GeoParams {
    double k;          // 2 pi / lambda
    double inv_lambda; // 1 / lambda
    double z0;
    double p2x, p2y;
    double x0, y0;     // destination window centre (extra pre-phase -k (x x0 + y y0) / r0)
    int nfx, nfy;      // fine grid
    int w;             // spreading width (cells)
    int log_tile_x, log_tile_y; // tile edges (cells), as powers of two
    int ntx, nty;      // tiles per axis
    int plane;         // 1: u_I = exp(i k d1) (cancels the -k d1 term exactly)
};

struct SpreadParams {
    int64_t n;         // source points (bound on the gathered index)
    int nfx, nfy, w, ntx, nty;
    int log_tile_x, log_tile_y, log_ntx;   // tile edges and tiles per row, as powers of two
    int log_panel;     // fine-grid panel width (columns stored contiguously per row), log2
    float beta_log2e;  // ES shape beta times log2(e), for exp2
};

// One batch of same-length FFTs.  In the first pass (along y) a workgroup
// transforms `batch` adjacent fine-grid columns; in the second pass (along x)
// it transforms `batch` rows of the intermediate array.
struct FftShape {
    int L;          // transform length, a power of two in [32, 16384]
    int batch;      // transforms per workgroup
};

// ---- one-dimensional (line) path -------------------------------------------------

// Scalars of a line plan.
struct LineGeo {
    double inv_lambda; // 1 / lambda
    double z0, p2, x0;
    int n, m, nf, log_nf, w;
    int plane;         // 1: u_I = exp(i k d1)
    double beta;       // ES shape
};

// Points of a line plan sorted by first footprint cell (ties by index).
struct LineBins {
    uint32_t *status;  // [1] bit 0: domain error
    uint32_t *first;   // [nf + 1] first sorted point whose footprint starts at cell c (or later)
    uint32_t *perm;    // [n] caller index of sorted point j
    uint32_t *cell;    // [n] its first footprint cell
    float2 *coef;      // [n][w] psi_a(offset_j) exp(i phi_j) for footprint cells a < w
};

constexpr int kLineMaxPoints = 16384;   // point index and first cell each fit 14 bits
constexpr int kLineKeyBits = 14;

hipError_t launch_line_setup(const LineGeo &g, const LineBins &b, const double *x, const double *d,
                             hipStream_t s);
hipError_t launch_line_forward(const LineGeo &g, const LineBins &b, const float2 *tw, const float2 *dd,
                               int batch, const float2 *u1, float2 *u2, hipStream_t s);

enum {
    STAGE_BIN = 0, STAGE_SCAN, STAGE_SCATTER, STAGE_SPREAD, STAGE_FFT1, STAGE_FFT2,   // forward
    STAGE_ADJ_FFT2, STAGE_ADJ_FFT1, STAGE_INTERP,                                      // adjoint
    NSTAGES
};

// ---- launchers (one per kernel family) ---------------------------------------
// clears both copies of status and cursor
hipError_t launch_bin_reset(const Binned &b, int ntiles, hipStream_t s);
// binning: the slab pass (bin_fill) or the count of the compact layout
// (bin_count), then the compact layout's scan and second pass, which return at
// once unless the status word says the compact layout is in use
hipError_t launch_bin_count(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                            const double *y, const double *d, hipStream_t s);
// crowded: slabs sized from a compact binning's counts (fewer workgroups at a time)
hipError_t launch_bin_fill(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                           const double *y, const double *d, bool crowded, hipStream_t s);
hipError_t launch_bin_scan(const Binned &b, int ntiles, hipStream_t s);
// (and, in every launch, clears next_status and next_cursor)
hipError_t launch_bin_scatter(const GeoParams &g, const Binned &b, int64_t n, int ntiles, const double *x,
                              const double *y, const double *d, hipStream_t s);
hipError_t launch_spread(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                         hipStream_t s);
// pass 1: columns of the fine grid (panel layout) -> mid (my x nfx, same panel layout)
hipError_t launch_fft_pass1(const FftShape &sh, int split16, const float2 *fine, float2 *mid,
                            const float2 *tw, const float2 *w16, int nfx, int my, hipStream_t s);
// pass 2: rows of mid (panels of 2^log_panel columns) -> u2[my][mx] with the
// deconvolution and destination phase
hipError_t launch_fft_pass2(const FftShape &sh, int log_panel, int split16, const float2 *mid,
                            float2 *u2, const float2 *tw, const float2 *w16, const float2 *dx,
                            const float2 *dy, int mx, int my, int accumulate, hipStream_t s);
// adjoint: rows of g2 (pre-corrected, zero-padded) -> mid (my x nfx, row-major)
hipError_t launch_fft_adj_rows(int len, int split16, const float2 *g2, float2 *mid, const float2 *tw,
                               const float2 *w16, const float2 *dx, const float2 *dy, int mx, int my,
                               hipStream_t s);
// adjoint: columns of mid (zero-padded) -> fine grid (panel layout)
hipError_t launch_fft_adj_cols(int len, int split16, const float2 *mid, float2 *fine,
                               const float2 *tw, const float2 *w16, int nfx, int my, hipStream_t s);
// adjoint of spreading: fine grid -> g1[n] (caller's order)
hipError_t launch_interp(const SpreadParams &p, const Binned &b, const float2 *fine, float2 *g1,
                         hipStream_t s);
// The library's fixed device scratch (ASF_STATIC_SCRATCH_BYTES on every device it
// runs on): its address on the current device, looked up on first use.
constexpr size_t kStaticScratchBytes = ASF_STATIC_SCRATCH_BYTES;
hipError_t static_scratch(void **out);

int fft_batch_pass1(int len);          // columns per workgroup in pass 1 (fine-grid panel width)
int fft_batch_pass2(int len);          // rows per workgroup in pass 2
size_t fft_lds_bytes(int len, int batch);
int fft_max_lds_bytes();

}  // namespace asf
