// One-dimensional form of the forward: a line source x1 with displacement
// d1(x1) onto a line of m destination pixels (the setting of the paper's
// profiles, Sec. 3), as a 1D type-1 NUFFT of Eq. (7)-(9) read for a surface that
// does not vary along y.
//
// The sizes are small (at most 16384 points, an oversampled line of at most
// 16384 cells), so one workgroup holds a whole problem:
//
//  * line_setup_kernel (one workgroup, at plan time): each point's FP64
//    pre-phase and frequency exactly as in the 2D geometry (phase in
//    revolutions s x^2 / 2 - s x x0 (- d / lambda without the plane wave),
//    s = 1 / (lambda r0), integer part removed in FP64, FP32 sincospi of the
//    remainder; frequency p2 x s wrapped to [0, 1), first footprint cell
//    c = ceil(g - w/2)), then a bitonic sort of the keys (c, index) in LDS and
//    the sorted records plus, per cell, the first point starting there.
//
//  * line_forward_kernel (one workgroup per field): each thread owns fine cells
//    and gathers the points whose footprint covers them from the w cells to
//    its left (a fixed order: no atomics, bitwise repeatable), writes the sum
//    to LDS in bit-reversed order, runs an in-place radix-2 FFT over the whole
//    line in LDS (FP32, twiddles from the FP64-built table) and multiplies the
//    kept modes by the deconvolution and destination phase.  The work is a few
//    microseconds of latency per field; batches of fields fill the chip.
#include <hip/hip_runtime.h>

#include "asf_internal.h"

namespace asf {
namespace {

constexpr int kLineThreads = 1024;

struct LinePoint {
    int c;          // first footprint cell, wrapped into [0, nf)
    float off;      // g - c - (w-1)/2
    float2 phase;   // exp(i phi)
    bool ok;
};

__device__ inline LinePoint line_point(const LineGeo &g, double x, double d) {
#pragma clang fp contract(off)
    LinePoint p;
    p.c = 0;
    p.off = 0.f;
    p.phase = make_float2(1.f, 0.f);
    const double r0 = g.z0 - d;
    p.ok = isfinite(x) && isfinite(d) && r0 > 0.0;
    if (!p.ok) return p;
    const double s = g.inv_lambda / r0;
    const double xi = g.p2 * x * s;
    double gg = (xi - floor(xi)) * (double)g.nf;
    if (gg >= (double)g.nf) gg -= (double)g.nf;
    int c = (int)ceil(gg - 0.5 * (double)g.w);
    p.off = (float)(gg - (double)c - 0.5 * (double)(g.w - 1));
    if (c < 0) c += g.nf;
    p.c = c;
    double rev = 0.5 * s * x * x;
    if (!g.plane) rev -= d * g.inv_lambda;
    rev -= x * g.x0 * s;
    const float t = (float)(rev - rint(rev));
    float sn, cs;
    sincospif(2.f * t, &sn, &cs);
    p.phase = make_float2(cs, sn);
    return p;
}

__global__ __launch_bounds__(kLineThreads) void line_setup_kernel(LineGeo g, LineBins b,
                                                                   const double *__restrict__ x,
                                                                   const double *__restrict__ d) {
    __shared__ uint32_t keys[kLineMaxPoints];
    const int n = g.n;
    int npad = 1;
    while (npad < n) npad <<= 1;
    const uint32_t mask = (1u << kLineKeyBits) - 1u;
    for (int i = threadIdx.x; i < npad; i += kLineThreads) {
        uint32_t key = 0xffffffffu;   // padding sorts last
        if (i < n) {
            const LinePoint p = line_point(g, x[i], d[i]);
            if (!p.ok) atomicOr(b.status, 1u);
            key = ((uint32_t)p.c << kLineKeyBits) | (uint32_t)i;
        }
        keys[i] = key;
    }
    __syncthreads();
    // bitonic sort, ascending; the keys are distinct (the index is in the low bits)
    for (int k = 2; k <= npad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < npad; i += kLineThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t a = keys[i], c = keys[l];
                    if ((a > c) == ((i & k) == 0)) {
                        keys[i] = c;
                        keys[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // sorted records; first[q] = first sorted point with cell >= q, for q in [0, nf]
    for (int j = threadIdx.x; j < n; j += kLineThreads) {
        const uint32_t key = keys[j];
        const uint32_t i = key & mask;
        const int c = (int)(key >> kLineKeyBits);
        const LinePoint p = line_point(g, x[i], d[i]);   // same function: same cell
        b.perm[j] = i;
        b.off[j] = p.off;
        b.phase[j] = p.phase;
        const int cprev = j == 0 ? -1 : (int)(keys[j - 1] >> kLineKeyBits);
        for (int q = cprev + 1; q <= c; ++q) b.first[q] = (uint32_t)j;
        if (j == n - 1)
            for (int q = c + 1; q <= g.nf; ++q) b.first[q] = (uint32_t)n;
    }
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(kLineThreads) void line_forward_kernel(LineGeo g, LineBins b,
                                                                     const float2 *__restrict__ tw,
                                                                     const float2 *__restrict__ dd,
                                                                     const float2 *__restrict__ u1,
                                                                     float2 *__restrict__ u2) {
    extern __shared__ float2 line[];   // nf cells
    const float2 *u = u1 + (size_t)blockIdx.x * g.n;
    const int nf = g.nf, w = g.w, lg = g.log_nf;
    const float two_over_w = 2.f / (float)w;
    const float centre = 0.5f * (float)(w - 1);

    // spreading as a gather: cell q is cell i = q - c of the footprints starting at c
    for (int q = threadIdx.x; q < nf; q += kLineThreads) {
        float ar = 0.f, ai = 0.f;
        for (int i = 0; i < w; ++i) {
            int c = q - i;
            if (c < 0) c += nf;
            const uint32_t j1 = b.first[c + 1];
            for (uint32_t j = b.first[c]; j < j1; ++j) {
                const float z = ((float)i - centre - b.off[j]) * two_over_w;
                const float a = 1.f - z * z;
                const float psi = a > 0.f ? exp2f(g.beta_log2e * (sqrtf(a) - 1.f)) : 0.f;
                const float2 v = cmul(u[b.perm[j]], b.phase[j]);
                ar = __builtin_fmaf(psi, v.x, ar);
                ai = __builtin_fmaf(psi, v.y, ai);
            }
        }
        line[__brev((unsigned)q) >> (32 - lg)] = make_float2(ar, ai);
    }
    __syncthreads();

    // in-place radix-2 decimation-in-time FFT, exp(-2 pi i k q / nf)
    for (int st = 1; st <= lg; ++st) {
        const int half = 1 << (st - 1);
        const int stride = nf >> st;
        for (int t = threadIdx.x; t < (nf >> 1); t += kLineThreads) {
            const int pos = t & (half - 1);
            const int a = ((t >> (st - 1)) << st) + pos;
            const float2 x0 = line[a];
            const float2 y0 = cmul(line[a + half], tw[pos * stride]);
            line[a] = make_float2(x0.x + y0.x, x0.y + y0.y);
            line[a + half] = make_float2(x0.x - y0.x, x0.y - y0.y);
        }
        __syncthreads();
    }

    // kept modes k = ix - m/2 at FFT index k mod nf, times the deconvolution and phase
    float2 *out = u2 + (size_t)blockIdx.x * g.m;
    for (int ix = threadIdx.x; ix < g.m; ix += kLineThreads) {
        const int k = ix - (g.m >> 1);
        out[ix] = cmul(line[k < 0 ? k + nf : k], dd[ix]);
    }
}

}  // namespace

hipError_t launch_line_setup(const LineGeo &g, const LineBins &b, const double *x, const double *d,
                             hipStream_t s) {
    if (g.n < 1 || g.n > kLineMaxPoints || g.nf < 2 || g.nf > (1 << kLineKeyBits)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(line_setup_kernel, dim3(1), dim3(kLineThreads), 0, s, g, b, x, d);
    return hipGetLastError();
}

hipError_t launch_line_forward(const LineGeo &g, const LineBins &b, const float2 *tw, const float2 *dd,
                               int batch, const float2 *u1, float2 *u2, hipStream_t s) {
    if (batch < 1 || g.nf < 2 || g.nf > (1 << kLineKeyBits) || (1 << g.log_nf) != g.nf)
        return hipErrorInvalidValue;
    const size_t lds = sizeof(float2) * (size_t)g.nf;
    static size_t enabled = 0;
    if (lds > 65536 && lds > enabled) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(line_forward_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        enabled = lds;
    }
    hipLaunchKernelGGL(line_forward_kernel, dim3(batch), dim3(kLineThreads), lds, s, g, b, tw, dd, u1, u2);
    return hipGetLastError();
}

}  // namespace asf
