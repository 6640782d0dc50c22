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
    // Slices of crowded tiles (written by every binning's scan, read by spreading and
    // interpolation).  A tile whose record count exceeds split_meta[0] is cut into
    // split[t] & 255 slices of consecutive records if split[t] != 0 (slots
    // split[t] >> 8 onward of the partial tiles); slot_owner[q] = t << 8 | slice
    // for the split_meta[1] slots in use.
    uint32_t *split;       // [ntiles]
    uint32_t *split_meta;  // [3] record threshold, slots in use, tiles no record reaches
    // Per tile, in tile order: 1 if some record reaches it, else 0 (written by every
    // binning's scan, on grids whose tiles may be cut).  Tiles flagged 0 may be left
    // unwritten by the spreading and the adjoint's column pass: the forward's column
    // pass then reads them as zeros, and no interpolation footprint reaches them.
    uint8_t *live;         // [ntiles]
    uint8_t *live_col;     // [ntx] per tile column: 1 if some tile of it is flagged 1
    uint32_t *slot_owner;  // [kSplitSlots]
    uint32_t *combine;     // [kSplitSlots] slices finished per split tile (zero between launches)
    unsigned long long *partial;   // [kSplitSlots][2][tile cells] integer sums of the slices (Re, Im),
                                   // in write-out order
};

// Crowded tiles.  A tile holding more than max(kSplitMinRecords, 2 R / slots)
// records (R: all records, slots: workgroups resident on the device at once) is
// cut into up to kSplitMaxSlices slices of at least kSliceMinRecords records, so
// a few tiles holding most of the points no longer run serially.  Every slice
// also reads all of its tile's records once (for the common scale), so slices
// are long: a workgroup's full batch of records (128^2 relief, four tiles of
// ~5,700 records: spread 0.062 ms with 256-record slices, 0.036 with 512, 0.033
// with 1024, 0.040 with 2048).
constexpr int kSplitSlots = 512;
constexpr int kSplitMaxSlices = 32;
constexpr uint32_t kSplitMinRecords = 2048;
constexpr uint32_t kSliceMinRecords = 1024;
constexpr uint32_t kNoSplit = 0xffffffffu;   // split_meta[0] when no tile is cut

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

// Workgroup blockIdx.x of a spreading or interpolation launch of ntiles + kSplitSlots
// workgroups: the tile it takes and its records [s0, s1); slice and slices (1 if
// the tile is not cut) and the first partial slot of the tile.  False if the
// workgroup has nothing to do (uniform over the workgroup).
__device__ inline bool tile_work(const Binned &b, int ntiles, int &t, uint32_t &slice, uint32_t &nsl,
                                 uint32_t &slot, uint32_t &s0, uint32_t &s1) {
    t = blockIdx.x;
    slice = 0;
    nsl = 1;
    slot = 0;
    if (t >= ntiles) {
        const uint32_t q = (uint32_t)(t - ntiles);
        if (q >= b.split_meta[1]) return false;
        const uint32_t own = b.slot_owner[q];
        slice = own & 255u;
        if (slice == 0) return false;   // slice 0 is the tile's own workgroup
        t = (int)(own >> 8);
    }
    tile_slots(b, t, s0, s1);
    if (s1 - s0 > b.split_meta[0]) {
        const uint32_t sp = b.split[t];
        if (sp) {
            nsl = sp & 255u;
            slot = sp >> 8;
            const uint32_t len = (s1 - s0 + nsl - 1) / nsl;
            const uint32_t a = s0 + min(s1 - s0, slice * len);
            s1 = a + min(s1 - a, len);
            s0 = a;
        }
    }
    return true;
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
    int split;         // 1: crowded tiles may be cut (launches take kSplitSlots more workgroups)
    int skip_dead;     // 1: tiles no record reaches are left unwritten
};

// Tile rows and columns of the largest fine grid (16384 cells a side, 64 x 32 tiles).
constexpr int kMaxTileRows = 512;
constexpr int kMaxTileCols = 256;

// The binning's per-tile flags (Binned::live, live_col) as the FFT passes take them.
// Forward: tiles flagged 0 were not written and are read as zeros, and the columns
// of a tile column with no flagged tile are neither transformed by the column pass
// nor read by the row pass (they are zeros); adjoint: the cells and columns are not
// needed.  flag NULL: every tile is written and read.
struct LiveTiles {
    const uint8_t *flag;   // [ty][tx]
    const uint8_t *col;    // [tx]
    int ntx, nty, log_tile_x, log_tile_y;
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
// the slab pass: one workgroup per point block, the blocks in a scattered order
hipError_t launch_bin_fill(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                           const double *y, const double *d, hipStream_t s);
// (and the slices of crowded tiles: slots = workgroups resident at once, 0 = never cut)
hipError_t launch_bin_scan(const Binned &b, int ntiles, int ntx, uint32_t slots, hipStream_t s);
// (and, in every launch, clears next_status and next_cursor)
hipError_t launch_bin_scatter(const GeoParams &g, const Binned &b, int64_t n, int ntiles, const double *x,
                              const double *y, const double *d, hipStream_t s);
hipError_t launch_spread(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                         hipStream_t s);
// pass 1: columns of the fine grid (panel layout) -> mid (my x nfx, same panel layout)
hipError_t launch_fft_pass1(const FftShape &sh, int split16, const float2 *fine, float2 *mid,
                            const float2 *tw, const float2 *w16, int nfx, int my, const LiveTiles &lt,
                            hipStream_t s);
// pass 2: rows of mid (panels of 2^log_panel columns) -> u2[my][mx] with the
// deconvolution and destination phase
hipError_t launch_fft_pass2(const FftShape &sh, int log_panel, int split16, const float2 *mid,
                            float2 *u2, const float2 *tw, const float2 *w16, const float2 *dx,
                            const float2 *dy, int mx, int my, int accumulate, const LiveTiles &lt,
                            hipStream_t s);
// adjoint: rows of g2 (pre-corrected, zero-padded) -> mid (my x nfx, row-major)
hipError_t launch_fft_adj_rows(int len, int split16, const float2 *g2, float2 *mid, const float2 *tw,
                               const float2 *w16, const float2 *dx, const float2 *dy, int mx, int my,
                               const LiveTiles &lt, hipStream_t s);
// adjoint: columns of mid (zero-padded) -> fine grid (panel layout)
hipError_t launch_fft_adj_cols(int len, int split16, const float2 *mid, float2 *fine,
                               const float2 *tw, const float2 *w16, int nfx, int my, const LiveTiles &lt,
                               hipStream_t s);
// adjoint of spreading: fine grid -> g1[n] (caller's order)
hipError_t launch_interp(const SpreadParams &p, const Binned &b, const float2 *fine, float2 *g1,
                         hipStream_t s);
// The library's fixed device scratch (ASF_STATIC_SCRATCH_BYTES on every device it
// runs on): its address on the current device, looked up on first use.
constexpr size_t kStaticScratchBytes = ASF_STATIC_SCRATCH_BYTES;
hipError_t static_scratch(void **out);

int fft_batch_pass1(int len);          // columns per workgroup in pass 1 (fine-grid panel width)
int fft_mid_panel(int len);            // columns per panel of pass 1's output (mid)
int fft_batch_pass2(int len);          // rows per workgroup in pass 2
size_t fft_lds_bytes(int len, int batch);
int fft_max_lds_bytes();

}  // namespace asf
