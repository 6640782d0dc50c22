// Spreading on gfx950: the "interpolation" half of the non-uniform FFT the
// paper evaluates Eq. (9) with (Sec. 2).  Each binned point carries
// c_j = u1_j exp(i phi_j) and adds c_j psi(l_x - g_x) psi(l_y - g_y) to the w x w
// fine cells around its position g (periodic), where psi is the
// exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)).
//
// One workgroup owns one tile of the fine grid.  Its bin lists every point whose
// footprint touches the tile, so the workgroup accumulates whole footprints
// into an LDS tile padded by w-1 cells on each side (no clipping), then writes
// only its own cells -- every fine cell is written exactly once with plain
// stores, no global atomics and no separate clear of the fine grid.
//
// Accumulation is in fixed point with LDS integer atomics: on gfx950 an LDS
// float atomic add runs about one lane at a time, the integer ones at full LDS
// rate.  A term t is made an integer by y = fma(a, k, 1.5 * 2^23): for
// |t| <= 2^22 the float y lies in [2^23, 2^24), where floats are the integers,
// so the FMA rounds the exact product to the nearest integer (ties to even:
// unbiased, which matters because a bias per term would add up coherently over
// ~1e9 terms at the lowest modes) and the bit pattern of y is
// 0x4B400000 + round(t).  One 64-bit integer add of a constant then removes the
// 0x4B400000 offsets.  The scale 2^e is set per tile as the largest e with
// 2^e M <= 2^22, M = max over the tile's points of |Re u1| + |Im u1| (a bound on
// |c_j|), so the rounding step is M 2^-22.  Two ways of holding a cell, chosen
// per tile from K = w^2 times the largest number of footprints that start in
// one cell (an upper bound on the terms any cell receives):
//   packed:  if K <= 511 no cell sum can leave int32 (511 * 2^22 < 2^31), and
//            one 64-bit word holds Re + 2^32 Im, so a single ds_add_u64 adds
//            both parts of a term (the carry of the low half into the high
//            half is undone exactly at unpacking);
//   split:   otherwise (dense tiles) Re and Im are separate 64-bit sums,
//            accumulated in two sweeps over the same LDS array.
// Integer addition is associative, so the spread is bitwise deterministic.
//
// Each thread keeps the global loads of several slots in flight at once; on
// this path the time goes to memory latency, not to the LDS atomics.
//
// The fine grid is stored in panels of `panel` adjacent columns: element
// (gx, gy) lives at ((gx / panel) * nfy + gy) * panel + gx % panel, so that the
// first FFT pass reads a panel of columns as one contiguous block.
#include "asf_internal.h"

namespace asf {
namespace {

constexpr int kTileXMax = 64;
constexpr int kTileYMax = 32;
constexpr int kThreads = 512;
constexpr int kBatch = 4;   // slots per thread with loads in flight together

__device__ inline float es_kernel(float z, float beta_log2e) {
    const float a = fmaxf(0.f, 1.f - z * z);
    return __builtin_amdgcn_exp2f(beta_log2e * (__builtin_amdgcn_sqrtf(a) - 1.f));
}

constexpr float kMagic = 12582912.f;             // 1.5 * 2^23
constexpr unsigned kMagicBits = 0x4B400000u;      // bit pattern of kMagic

constexpr unsigned long long kMagic1 = kMagicBits;
constexpr unsigned long long kMagic2 = ((unsigned long long)kMagicBits << 32) | kMagicBits;

// round(a k) as a 64-bit two's-complement integer, for |a k| <= 2^22
__device__ inline unsigned long long term1(float a, float k) {
    return (unsigned long long)__float_as_uint(__builtin_fmaf(a, k, kMagic)) - kMagic1;
}

// round(re) + 2^32 round(im) modulo 2^64, for |re|, |im| <= 2^22
__device__ inline unsigned long long term(float ar, float ai, float k) {
    const float yr = __builtin_fmaf(ar, k, kMagic);
    const float yi = __builtin_fmaf(ai, k, kMagic);
    return (((unsigned long long)__float_as_uint(yi) << 32) | __float_as_uint(yr)) - kMagic2;
}

__device__ inline void unpack2(unsigned long long v, int &re, int &im) {
    re = (int)(unsigned)(v & 0xffffffffull);
    im = (int)(unsigned)((v - (unsigned long long)(long long)re) >> 32);
}

__device__ inline float block_max(float v, float *scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmaxf(s, scratch[i]);
    return s;
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

template <int W>
__global__ void __launch_bounds__(kThreads) spread_kernel(SpreadParams p, Binned b,
                                                          const float2 *__restrict__ u1,
                                                          float2 *__restrict__ fine) {
    constexpr int PAD = W - 1;
    constexpr int CELLS = (kTileXMax + 2 * PAD) * (kTileYMax + 2 * PAD);
    constexpr int STARTS = (kTileXMax + PAD) * (kTileYMax + PAD);
    constexpr int B = kBatch;
    __shared__ unsigned long long acc[CELLS];
    __shared__ int starts[STARTS];                 // footprint starts per padded cell
    __shared__ float scratch[kThreads / 64];

    const int t = blockIdx.x;
    const int ty = t >> p.log_ntx, tx = t & ((1 << p.log_ntx) - 1);
    const int tsx = 1 << p.log_tile_x, tsy = 1 << p.log_tile_y;
    const int x0 = tx << p.log_tile_x, y0 = ty << p.log_tile_y;
    const int pwx = tsx + 2 * PAD, pwy = tsy + 2 * PAD;   // padded tile; pwx = LDS row stride
    const int swx = tsx + PAD, swy = tsy + PAD;           // start positions per axis
    const int hix = swx - 1, hiy = swy - 1;
    const int nt = blockDim.x;
    for (int i = threadIdx.x; i < pwx * pwy; i += nt) acc[i] = 0ull;
    for (int i = threadIdx.x; i < swx * swy; i += nt) starts[i] = 0;
    __syncthreads();

    // pass 1: largest |Re u1| + |Im u1| and the count of footprint starts per
    // position; B slots per thread have their loads in flight together
    const uint32_t s0 = b.tile_start[t], s1 = b.tile_start[t + 1];
    float big = 0.f;
    for (uint32_t base = s0 + threadIdx.x; base < s1; base += B * nt) {
        uint32_t j[B], cell[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint32_t s = base + k * nt;
            const bool in = s < s1;
            j[k] = in ? b.perm[s] : 0xffffffffu;
            cell[k] = in ? b.cell[s] : 0u;
        }
        float2 u[B];
#pragma unroll
        for (int k = 0; k < B; ++k) u[k] = j[k] < p.n ? u1[j[k]] : make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < B; ++k) {
            int px, py;
            if (j[k] < p.n && local_start(cell[k], x0, y0, PAD, hix, hiy, p.nfx, p.nfy, px, py)) {
                big = fmaxf(big, fabsf(u[k].x) + fabsf(u[k].y));
                atomicAdd(&starts[py * swx + px], 1);
            }
        }
    }
    big = block_max(big, scratch);   // contains a barrier: starts[] is complete
    int most = 0;                    // most footprint starts in one cell
    for (int i = threadIdx.x; i < swx * swy; i += nt) most = max(most, starts[i]);
    const float kbound = (float)(W * W) * block_max((float)most, scratch);
    int e = 0;
    if (big > 0.f) {
        int em;
        frexpf(big, &em);                   // big <= 2^em
        e = 22 - em;
    }
    const bool packed = kbound <= 511.f;
    e = max(-120, min(e, 120));
    const float scale = ldexpf(1.f, e);
    const double unscale = ldexp(1.0, -e);

    // pass 2: accumulate every footprint.  Packed tiles need one sweep; split
    // (dense) tiles sweep twice over one 64-bit array, Re first, then Im.
    constexpr float kz = 2.f / (float)W;
    constexpr float half = 0.5f * (float)(W - 1);
    const bool fold_x = p.nfx < pwx, fold_y = p.nfy < pwy;
    const int C = 1 << p.log_panel;
    const int ncell = tsx * tsy;
    const int sweeps = packed ? 1 : 2;
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (uint32_t base = s0 + threadIdx.x; base < s1; base += B * nt) {
            uint32_t j[B], cell[B];
            float2 fr[B], ph[B];
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const uint32_t s = base + k * nt;
                const bool in = s < s1;
                j[k] = in ? b.perm[s] : 0xffffffffu;
                cell[k] = in ? b.cell[s] : 0u;
                fr[k] = in ? b.frac[s] : make_float2(0.f, 0.f);
                ph[k] = in ? b.phase[s] : make_float2(0.f, 0.f);
            }
            float2 u[B];
#pragma unroll
            for (int k = 0; k < B; ++k) u[k] = j[k] < p.n ? u1[j[k]] : make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < B; ++k) {
                int px, py;
                if (!(j[k] < p.n && local_start(cell[k], x0, y0, PAD, hix, hiy, p.nfx, p.nfy, px, py))) continue;
                const float cr = (u[k].x * ph[k].x - u[k].y * ph[k].y) * scale;
                const float ci = (u[k].x * ph[k].y + u[k].y * ph[k].x) * scale;
                // split sweep 0 adds Re, sweep 1 adds Im, each into the low half
                const float c0 = packed ? cr : (sweep == 0 ? cr : ci);
                float kx[W];
#pragma unroll
                for (int i = 0; i < W; ++i) kx[i] = es_kernel(((float)i - half - fr[k].x) * kz, p.beta_log2e);
                unsigned long long *row = acc + py * pwx + px;
#pragma unroll
                for (int jy = 0; jy < W; ++jy) {
                    const float ky = es_kernel(((float)jy - half - fr[k].y) * kz, p.beta_log2e);
                    const float ar = c0 * ky, ai = ci * ky;
                    if (packed) {
#pragma unroll
                        for (int i = 0; i < W; ++i) atomicAdd(row + jy * pwx + i, term(ar, ai, kx[i]));
                    } else {
#pragma unroll
                        for (int i = 0; i < W; ++i) atomicAdd(row + jy * pwx + i, term1(ar, kx[i]));
                    }
                }
            }
        }
        __syncthreads();

        // read back the tile's own cells (in the order they are written out);
        // on axes where the whole grid is narrower than the padded tile, fold
        // the wrapped halo back in
        for (int i = threadIdx.x; i < ncell; i += nt) {
            const int c = i & (C - 1);
            const int rest = i >> p.log_panel;
            const int ly = rest & (tsy - 1);
            const int q = rest >> p.log_tile_y;
            const int lx = (q << p.log_panel) + c;
            unsigned long long v = 0ull;
            if (!fold_x && !fold_y) {
                v = acc[(ly + PAD) * pwx + lx + PAD];
            } else {
                for (int oy = ly + PAD - 2 * p.nfy; oy < pwy; oy += p.nfy) {
                    if (oy < 0 || (!fold_y && oy != ly + PAD)) continue;
                    for (int ox = lx + PAD - 2 * p.nfx; ox < pwx; ox += p.nfx) {
                        if (ox < 0 || (!fold_x && ox != lx + PAD)) continue;
                        v += acc[oy * pwx + ox];
                    }
                }
            }
            const int gx = x0 + lx, gy = y0 + ly;
            float2 *dst = fine + ((((size_t)(gx >> p.log_panel) * p.nfy + gy) << p.log_panel) + c);
            if (packed) {
                int sr, si;
                unpack2(v, sr, si);
                *dst = make_float2((float)((double)sr * unscale), (float)((double)si * unscale));
            } else {
                // split tiles: sweep 0 writes the real part, sweep 1 the imaginary part
                reinterpret_cast<float *>(dst)[sweep] = (float)((double)(long long)v * unscale);
            }
        }
        if (sweep + 1 < sweeps) {
            __syncthreads();
            for (int i = threadIdx.x; i < pwx * pwy; i += nt) acc[i] = 0ull;
            __syncthreads();
        }
    }
}

template <int W>
hipError_t launch_w(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                    hipStream_t s) {
    const int ntiles = p.ntx * p.nty;
    hipLaunchKernelGGL(spread_kernel<W>, dim3(ntiles), dim3(kThreads), 0, s, p, b, u1, fine);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_spread(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                         hipStream_t s) {
    if ((1 << p.log_tile_x) > kTileXMax || (1 << p.log_tile_y) > kTileYMax) return hipErrorInvalidValue;
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

}  // namespace asf
