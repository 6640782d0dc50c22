// Spreading on gfx950: the "interpolation" half of the non-uniform FFT the
// paper evaluates Eq. (9) with (Sec. 2).  Each binned point carries
// c_j = u1_j exp(i phi_j) and adds c_j psi(l_x - g_x) psi(l_y - g_y) to the w x w
// fine cells around its position g (periodic), where psi is the
// exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)).
//
// One workgroup owns one tile of the fine grid: it zeroes the tile in LDS,
// accumulates every point listed in the tile's bin (its own points and the
// neighbours whose footprint reaches in) with LDS float atomics, and writes the
// whole tile back with plain stores -- no global atomics, and every fine cell is
// written exactly once, so no separate clear of the fine grid is needed.
//
// The fine grid is stored in panels of `panel` adjacent columns: element
// (gx, gy) lives at ((gx / panel) * nfy + gy) * panel + gx % panel, so that the
// first FFT pass reads a panel of columns as one contiguous block.
#include "asf_internal.h"

namespace asf {
namespace {

constexpr int kTileMax = 64;
constexpr int kRowStride = kTileMax + 1;  // odd row stride spreads LDS banks

__device__ inline float es_kernel(float z, float beta_log2e) {
    const float a = fmaxf(0.f, 1.f - z * z);
    return __builtin_amdgcn_exp2f(beta_log2e * (__builtin_sqrtf(a) - 1.f));
}

template <int W>
__global__ void __launch_bounds__(256) spread_kernel(SpreadParams p, Binned b,
                                                     const float2 *__restrict__ u1,
                                                     float2 *__restrict__ fine) {
    __shared__ float tre[kTileMax * kRowStride];
    __shared__ float tim[kTileMax * kRowStride];
    const int t = blockIdx.x;
    const int ty = t / p.ntx, tx = t - ty * p.ntx;
    const int x0 = tx * p.tile, y0 = ty * p.tile;
    const int ts = p.tile;
    for (int i = threadIdx.x; i < kTileMax * kRowStride; i += blockDim.x) {
        tre[i] = 0.f;
        tim[i] = 0.f;
    }
    __syncthreads();

    const uint32_t s0 = b.tile_start[t], s1 = b.tile_start[t + 1];
    constexpr float scale = 2.f / (float)W;
    constexpr float half = 0.5f * (float)(W - 1);
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const uint32_t j = b.perm[s];
        if (j >= p.n) continue;   // never gather outside u1, whatever a slot holds
        const uint32_t cell = b.cell[s];
        const float2 fr = b.frac[s];
        const float2 ph = b.phase[s];
        const float2 u = u1[j];
        const float cr = u.x * ph.x - u.y * ph.y;
        const float ci = u.x * ph.y + u.y * ph.x;
        int ox = (int)(cell & 0xffffu) - x0;
        if (ox < 0) ox += p.nfx;
        int oy = (int)(cell >> 16) - y0;
        if (oy < 0) oy += p.nfy;
        float kx[W];
#pragma unroll
        for (int i = 0; i < W; ++i) kx[i] = es_kernel(((float)i - half - fr.x) * scale, p.beta_log2e);
#pragma unroll
        for (int jy = 0; jy < W; ++jy) {
            int ly = oy + jy;
            if (ly >= p.nfy) ly -= p.nfy;
            if (ly < ts) {
                const float ky = es_kernel(((float)jy - half - fr.y) * scale, p.beta_log2e);
                const float ar = cr * ky, ai = ci * ky;
                float *rre = tre + ly * kRowStride;
                float *rim = tim + ly * kRowStride;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    int lx = ox + i;
                    if (lx >= p.nfx) lx -= p.nfx;
                    if (lx < ts) {
                        atomicAdd(rre + lx, ar * kx[i]);
                        atomicAdd(rim + lx, ai * kx[i]);
                    }
                }
            }
        }
    }
    __syncthreads();

    // write the tile: panel by panel, each panel's rows contiguous in memory
    const int C = p.panel;
    const int n = ts * ts;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int c = i % C;
        const int rest = i / C;
        const int ly = rest % ts;
        const int q = rest / ts;
        const int lx = q * C + c;
        const int gx = x0 + lx, gy = y0 + ly;
        fine[((size_t)(gx / C) * p.nfy + gy) * C + c] =
            make_float2(tre[ly * kRowStride + lx], tim[ly * kRowStride + lx]);
    }
}

template <int W>
hipError_t launch_w(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                    hipStream_t s) {
    const int ntiles = p.ntx * p.nty;
    hipLaunchKernelGGL(spread_kernel<W>, dim3(ntiles), dim3(256), 0, s, p, b, u1, fine);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_spread(const SpreadParams &p, const Binned &b, const float2 *u1, float2 *fine,
                         hipStream_t s) {
    if (p.tile > kTileMax) return hipErrorInvalidValue;
    switch (p.w) {
        case 2: return launch_w<2>(p, b, u1, fine, s);
        case 3: return launch_w<3>(p, b, u1, fine, s);
        case 4: return launch_w<4>(p, b, u1, fine, s);
        case 5: return launch_w<5>(p, b, u1, fine, s);
        case 6: return launch_w<6>(p, b, u1, fine, s);
        case 7: return launch_w<7>(p, b, u1, fine, s);
        case 8: return launch_w<8>(p, b, u1, fine, s);
        case 9: return launch_w<9>(p, b, u1, fine, s);
        case 10: return launch_w<10>(p, b, u1, fine, s);
        case 11: return launch_w<11>(p, b, u1, fine, s);
        case 12: return launch_w<12>(p, b, u1, fine, s);
        case 13: return launch_w<13>(p, b, u1, fine, s);
        case 14: return launch_w<14>(p, b, u1, fine, s);
        case 15: return launch_w<15>(p, b, u1, fine, s);
        case 16: return launch_w<16>(p, b, u1, fine, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace asf
