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
// Accumulation is in 64-bit fixed point with LDS integer atomics.  On gfx950 an
// LDS float atomic add is executed about one lane at a time while the integer
// ones run at full LDS rate.  Each term is formed exactly as an integer:
//   A = round(Re/Im(c_j) psi_y 2^a)   (|A| <= 2^22, per point and row)
//   K = round(psi_x 2^22)             (per point and column)
//   A K                               (48-bit product: v_mul_i32_i24 + v_mul_hi_i32_i24)
// and added with ds_add_u64.  The exponent a is set per tile from
// M = max over its points of |Re u1| + |Im u1|, so 2^a M <= 2^22: the rounding of
// A and K is 2^-22 of the tile's largest point and of the kernel peak, about
// the size of FP32 rounding, whatever the number of points in the tile.  Sums
// stay below 2^62 for tiles of up to 2^18 points (a is lowered beyond that).
// Integer addition is associative, so the spread is bitwise deterministic.
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

__device__ inline float es_kernel(float z, float beta_log2e) {
    const float a = fmaxf(0.f, 1.f - z * z);
    return __builtin_amdgcn_exp2f(beta_log2e * (__builtin_sqrtf(a) - 1.f));
}

// round to nearest, ties to even: unbiased for either sign (a round-half-up
// conversion would add a positive bias to every term, which piles up at the
// low modes)
__device__ inline int round_even(float x) { return (int)__builtin_rintf(x); }

// exact product of two values known to fit in 24 signed bits
__device__ inline unsigned long long mul24_wide(int a, int k) {
    const int as = (a << 8) >> 8, ks = (k << 8) >> 8;
    return (unsigned long long)((long long)as * (long long)ks);
}

__device__ inline float block_max(float v, float *scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[wave] = v;
    __syncthreads();
    float s = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmaxf(s, scratch[i]);
    return s;
}

template <int W>
__global__ void __launch_bounds__(kThreads) spread_kernel(SpreadParams p, Binned b,
                                                          const float2 *__restrict__ u1,
                                                          float2 *__restrict__ fine) {
    constexpr int PAD = W - 1;
    constexpr int CELLS = (kTileXMax + 2 * PAD) * (kTileYMax + 2 * PAD);
    __shared__ unsigned long long acc_re[CELLS];
    __shared__ unsigned long long acc_im[CELLS];
    __shared__ float scratch[kThreads / 64];

    const int t = blockIdx.x;
    const int ty = t / p.ntx, tx = t - ty * p.ntx;
    const int tsx = p.tile_x, tsy = p.tile_y;
    const int x0 = tx * tsx, y0 = ty * tsy;
    const int pwx = tsx + 2 * PAD, pwy = tsy + 2 * PAD;   // padded tile; pwx = LDS row stride
    for (int i = threadIdx.x; i < pwx * pwy; i += blockDim.x) {
        acc_re[i] = 0ull;
        acc_im[i] = 0ull;
    }

    // fixed-point exponent from the largest |Re u1| + |Im u1| among the tile's points
    const uint32_t s0 = b.tile_start[t], s1 = b.tile_start[t + 1];
    float big = 0.f;
#pragma unroll 4
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const uint32_t j = b.perm[s];
        if (j < p.n) {
            const float2 u = u1[j];
            big = fmaxf(big, fabsf(u.x) + fabsf(u.y));
        }
    }
    big = block_max(big, scratch);
    int em = 0;
    if (big > 0.f) frexpf(big, &em);                     // big <= 2^em
    int cnt_bits = 0;
    while (cnt_bits < 31 && (1u << cnt_bits) < (s1 - s0)) ++cnt_bits;
    int a = 22 - em - (cnt_bits > 18 ? cnt_bits - 18 : 0);
    a = max(-100, min(a, 100));
    const float scale_a = ldexpf(1.f, a);
    const double unscale = ldexp(1.0, -(a + 22));

    constexpr float kz = 2.f / (float)W;
    constexpr float half = 0.5f * (float)(W - 1);
    const int hix = tsx + PAD - 1, hiy = tsy + PAD - 1;   // largest valid padded start
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const uint32_t j = b.perm[s];
        if (j >= p.n) continue;   // never gather outside u1, whatever a slot holds
        const uint32_t cell = b.cell[s];
        int px = (int)(cell & 0xffffu) - x0 + PAD;
        if (px < 0) px += p.nfx;
        else if (px > hix) px -= p.nfx;
        int py = (int)(cell >> 16) - y0 + PAD;
        if (py < 0) py += p.nfy;
        else if (py > hiy) py -= p.nfy;
        if (px < 0 || px > hix || py < 0 || py > hiy) continue;
        const float2 fr = b.frac[s];
        const float2 ph = b.phase[s];
        const float2 u = u1[j];
        const float cr = (u.x * ph.x - u.y * ph.y) * scale_a;
        const float ci = (u.x * ph.y + u.y * ph.x) * scale_a;
        int kx[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            kx[i] = round_even(es_kernel(((float)i - half - fr.x) * kz, p.beta_log2e) * 4194304.f);
        unsigned long long *rre = acc_re + py * pwx + px;
        unsigned long long *rim = acc_im + py * pwx + px;
#pragma unroll
        for (int jy = 0; jy < W; ++jy) {
            const float ky = es_kernel(((float)jy - half - fr.y) * kz, p.beta_log2e);
            const int ar = round_even(cr * ky), ai = round_even(ci * ky);
#pragma unroll
            for (int i = 0; i < W; ++i) {
                atomicAdd(rre + jy * pwx + i, mul24_wide(ar, kx[i]));
                atomicAdd(rim + jy * pwx + i, mul24_wide(ai, kx[i]));
            }
        }
    }
    __syncthreads();

    // write the tile's own cells, panel by panel; on axes where the whole grid
    // is narrower than the padded tile, fold the wrapped halo back in
    const bool fold_x = p.nfx < pwx, fold_y = p.nfy < pwy;
    const int C = p.panel;
    const int n = tsx * tsy;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int c = i % C;
        const int rest = i / C;
        const int ly = rest % tsy;
        const int q = rest / tsy;
        const int lx = q * C + c;
        long long sr = 0, si = 0;
        if (!fold_x && !fold_y) {
            const int at = (ly + PAD) * pwx + lx + PAD;
            sr = (long long)acc_re[at];
            si = (long long)acc_im[at];
        } else {
            for (int oy = ly + PAD - 2 * p.nfy; oy < pwy; oy += p.nfy) {
                if (oy < 0 || (!fold_y && oy != ly + PAD)) continue;
                for (int ox = lx + PAD - 2 * p.nfx; ox < pwx; ox += p.nfx) {
                    if (ox < 0 || (!fold_x && ox != lx + PAD)) continue;
                    sr += (long long)acc_re[oy * pwx + ox];
                    si += (long long)acc_im[oy * pwx + ox];
                }
            }
        }
        const int gx = x0 + lx, gy = y0 + ly;
        fine[((size_t)(gx / C) * p.nfy + gy) * C + c] =
            make_float2((float)((double)sr * unscale), (float)((double)si * unscale));
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
    if (p.tile_x > kTileXMax || p.tile_y > kTileYMax) return hipErrorInvalidValue;
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
