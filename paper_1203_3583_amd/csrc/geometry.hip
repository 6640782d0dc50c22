// Geometry stage on gfx950: the FP64 pre-phase of Eq. (8) and the per-point
// frequencies of Eq. (9) (Sec. 2), and binning of the points into fine-grid
// tiles for the spreading kernel.
//
// For point j with r0 = z0 - d1 (Eq. (4)):
//   phi_j  = k (-d_j + |x_j|^2 / (2 r0_j)) + arg u_I,j        (pre-phase, Eq. (7)/(8))
//   xi_j   = p2 x_j / (lambda r0_j)                           (cycles per destination pixel)
// With the normal plane wave u_I = exp(i k d1) the -k d1 term and the incident
// phase cancel exactly, so the kernel forms phi = k |x|^2 / (2 r0) directly and
// never builds the ~1e4 rad intermediate.  phi is reduced mod 2 pi in FP64
// before the FP64 sincos; xi is wrapped to [0, 1) (exp(-2 pi i m xi) is
// 1-periodic in xi for integer m) and scaled to the fine grid, g = xi * nf.
// The footprint of the spreading kernel starts at cell l0 = ceil(g - w/2); the
// FP32 offset g - l0 - (w-1)/2 lies in (-1/2, 1/2], so its rounding error is at
// most 2^-26 cell however large the phase was.
//
// Binning: each point is listed once in every tile its w x w footprint touches
// (1, 2 or 4 tiles), so the spreading kernel can own its tile outright and write
// it with plain stores.  Counting and scattering aggregate per wavefront: the
// lanes are grouped by tile without memory traffic, then one lane per group
// issues the atomic -- all groups' atomics in the same instruction, so a wave
// waits for one round trip rather than one per tile.
#include "asf_internal.h"

namespace asf {
namespace {

constexpr double kTwoPiHi = 6.283185307179586;        // 2 pi rounded to FP64
constexpr double kTwoPiLo = 2.4492935982947064e-16;   // 2 pi - kTwoPiHi

struct PointTiles {
    int n;        // tiles touched (0 if the point is invalid)
    int key[4];   // tile indices ty * ntx + tx
    int l0x, l0y; // first footprint cell, wrapped into the fine grid
    float fx, fy; // offsets in (-1/2, 1/2]
    double r0;
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

__device__ inline int axis_tiles(int l0, int nf, int w, int tile, int *t) {
    int last = l0 + w - 1;
    if (last >= nf) last -= nf;
    t[0] = l0 / tile;
    t[1] = last / tile;
    return t[1] != t[0] ? 2 : 1;
}

__device__ inline PointTiles point_tiles(const GeoParams &g, double x, double y, double d) {
#pragma clang fp contract(off)
    PointTiles p;
    p.n = 0;
    p.l0x = p.l0y = 0;
    p.fx = p.fy = 0.f;
    p.r0 = g.z0 - d;
    if (!(p.r0 > 0.0) || !isfinite(x) || !isfinite(y) || !isfinite(d)) return p;
    const double s = g.inv_lambda / p.r0;
    axis_cell(g.p2x * x * s, g.nfx, g.w, p.l0x, p.fx);
    axis_cell(g.p2y * y * s, g.nfy, g.w, p.l0y, p.fy);
    int tx[2], ty[2];
    const int nx = axis_tiles(p.l0x, g.nfx, g.w, g.tile_x, tx);
    const int ny = axis_tiles(p.l0y, g.nfy, g.w, g.tile_y, ty);
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b) p.key[p.n++] = ty[a] * g.ntx + tx[b];
    return p;
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
    WaveGroup g;
    g.leader = lane;
    g.rank = 0u;
    g.size = 0u;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int lkey = __shfl(key, leader);
        const uint64_t mask = __ballot(active && key == lkey) & todo;
        if ((mask >> lane) & 1ull) {
            g.leader = leader;
            g.rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            if (lane == leader) g.size = (uint32_t)__popcll(mask);
        }
        todo &= ~mask;
    }
    return g;
}

__global__ void __launch_bounds__(256) bin_reset_kernel(Binned b, int ntiles) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntiles) b.cursor[i] = 0u;
    if (i == 0) b.status[0] = 0u;
}

__global__ void __launch_bounds__(256) bin_count_kernel(GeoParams g, Binned b, int64_t n,
                                                        const double *__restrict__ x,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ d) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    PointTiles p;
    p.n = 0;
    if (j < n) {
        p = point_tiles(g, x[j], y[j], d[j]);
        if (p.n == 0) atomicOr(b.status, 1u);
    }
    // one non-returning atomic per distinct tile per wave and replica
    for (int r = 0; r < 4; ++r) {
        const bool act = r < p.n;
        const WaveGroup grp = wave_group(act ? p.key[r] : 0, act);
        if (act && grp.leader == __lane_id()) atomicAdd(&b.cursor[p.key[r]], grp.size);
    }
}

// Exclusive scan of the per-tile counts by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) bin_scan_kernel(Binned b, int ntiles) {
    __shared__ uint32_t sums[1024];
    const int t = threadIdx.x;
    const int per = (ntiles + 1023) / 1024;
    const int lo = min(t * per, ntiles), hi = min(lo + per, ntiles);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += b.cursor[i];
    sums[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? sums[t - off] : 0u;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    uint32_t run = t ? sums[t - 1] : 0u;
    for (int i = lo; i < hi; ++i) {
        const uint32_t c = b.cursor[i];
        b.tile_start[i] = run;
        b.cursor[i] = run;
        run += c;
    }
    if (t == 1023) b.tile_start[ntiles] = sums[1023];
}

__global__ void __launch_bounds__(256) bin_scatter_kernel(GeoParams g, Binned b, int64_t n,
                                                          const double *__restrict__ x,
                                                          const double *__restrict__ y,
                                                          const double *__restrict__ d) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    PointTiles p;
    p.n = 0;
    float2 ph = make_float2(0.f, 0.f);
    if (j < n) {
        const double xj = x[j], yj = y[j], dj = d[j];
        p = point_tiles(g, xj, yj, dj);
        if (p.n > 0) {
            double q = (xj * xj + yj * yj) / (2.0 * p.r0);
            if (!g.plane) q -= dj;
            const double phi = g.k * q;
            const double nrev = rint(phi / kTwoPiHi);
            double red = fma(-nrev, kTwoPiHi, phi);
            red = fma(-nrev, kTwoPiLo, red);
            double sn, cs;
            sincos(red, &sn, &cs);
            ph = make_float2((float)cs, (float)sn);
        }
    }
    const uint32_t cell = (uint32_t)p.l0x | ((uint32_t)p.l0y << 16);
    // group the four replica keys first, then let the leaders reserve their
    // groups' slots with atomics that are all in flight at once
    WaveGroup grp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) grp[r] = wave_group(r < p.n ? p.key[r] : 0, r < p.n);
    uint32_t base[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        base[r] = (r < p.n && grp[r].leader == __lane_id()) ? atomicAdd(&b.cursor[p.key[r]], grp[r].size) : 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const bool act = r < p.n;
        const int key = act ? p.key[r] : 0;
        const uint32_t slot = __shfl(base[r], grp[r].leader) + grp[r].rank;
        if (act) {
            if (slot < b.tile_start[key + 1]) {
                b.cell[slot] = cell;
                b.frac[slot] = make_float2(p.fx, p.fy);
                b.phase[slot] = ph;
                b.perm[slot] = (uint32_t)j;
            } else {
                atomicOr(b.status, 2u);
            }
        }
    }
}

}  // namespace

hipError_t launch_bin_reset(const Binned &b, int ntiles, hipStream_t s) {
    const int blocks = (ntiles + 255) / 256;
    hipLaunchKernelGGL(bin_reset_kernel, dim3(blocks), dim3(256), 0, s, b, ntiles);
    return hipGetLastError();
}

hipError_t launch_bin_count(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                            const double *y, const double *d, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, b, n, x, y, d);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Binned &b, int ntiles, hipStream_t s) {
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(1024), 0, s, b, ntiles);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const GeoParams &g, const Binned &b, int64_t n, const double *x,
                              const double *y, const double *d, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, b, n, x, y, d);
    return hipGetLastError();
}

}  // namespace asf
