// Host-side plan arithmetic of the library: parameter checks, the workspace
// layouts, and the FP64 tables the kernels read (Gauss-Legendre nodes, the
// spreading kernel's Fourier transform, the FFT stage twiddles).  Plain C++ with
// no HIP dependency, so that it can be built and exercised on its own (under
// the address and undefined-behaviour sanitizers in the CPU tests).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "asf.h"

namespace asf {
namespace host {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr int kTileXMax = 64;      // spreading tile: 64 x 32 fine cells
constexpr int kTileYMax = 32;
constexpr int kLineMaxPoints = 16384;
constexpr int kSplitSlotsHost = 512;   // partial tiles of cut crowded tiles

// A complex value as two FP32 numbers, laid out like HIP's float2.
struct Cf {
    float re, im;
};

// Record a failure message for asf_last_error (thread-local) and return code.
int fail(int code, const char *fmt, ...);
const char *last_error();

size_t align_up(size_t v);
bool is_pow2(int v);
int log2i(int v);

// Workspace of a 2D plan: byte offsets of its segments (256-byte aligned).
struct Layout {
    int64_t n;
    int mx, my, nfx, nfy, w, tile_x, tile_y, ntx, nty, ntiles;
    double beta;
    int64_t slot_cap;
    size_t off_status, off_tile_start, off_cursor, off_slab, off_cell, off_frac, off_phase, off_perm;
    size_t off_status2, off_cursor2;   // the counters' second copy
    size_t off_fine, off_mid, off_dx, off_dy, off_twx, off_twy, off_w16;
    // crowded tiles cut into slices (only grids wider than a tile plus its halo)
    bool split;
    size_t off_split, off_split_meta, off_slot_owner, off_combine, off_partial;
    size_t off_live;   // per-tile flags of the last spread (u8 [ntx][nty])
    size_t total;
};

int check_params(int64_t n, const asf_params *p);
// spreading width w for a requested tolerance: ceil(log10(1 / tol)) + 2 in [2, 9]
int spread_width(double tol);
int make_layout(int64_t n, const asf_params *p, Layout &L);

// Workspace of a line plan.
struct LineLayout {
    int n, m, nf, w;
    double beta;
    size_t off_status, off_first, off_perm, off_cell, off_coef, off_tw, off_dd, total;
};
int make_line_layout(int64_t n, const asf_line_params *p, LineLayout &L);

// n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wq);
// Fourier transform of the spreading kernel at modes 0 .. nmodes_half of an nf grid.
std::vector<double> psi_hat(int nmodes_half, int nf, int w, double beta);
// complex entries of one length's stage twiddle tables
size_t fft_twiddle_entries(int len);
// the stage twiddle tables of a length-len FFT, in the order the kernels read them
std::vector<Cf> stage_twiddles(int len);
// a phase argument (rad) reduced to [-pi, pi] in FP64
double reduce(double a);

}  // namespace host
}  // namespace asf
