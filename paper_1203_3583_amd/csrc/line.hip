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
//    c = ceil(g - w/2)), then a bitonic sort of the keys (c, index) in LDS, and
//    per sorted point its caller index and its w spreading coefficients
//    psi_i(offset) exp(i phi) (kernel values in FP64, rounded once), plus, per
//    cell, the first point starting there.
//
//  * line_forward_kernel (one 256-thread workgroup per field): each thread owns
//    fine cells and gathers the points whose footprint covers them -- those
//    starting in the w cells up to its own, one contiguous run of the sorted
//    list -- one complex multiply-add per (cell, point) pair, in a fixed order
//    (no atomics, bitwise repeatable); the sums go to LDS in
//    bit-reversed order; an in-place FFT over the whole line follows in LDS
//    (FP32, FP64-built twiddles), two radix-2 levels per pass (radix-4
//    butterflies, half the barriers), and the kept modes are multiplied by the
//    deconvolution and destination phase.  Small workgroups let several fields
//    share a CU and hide each other's barriers.
#include <hip/hip_runtime.h>

#include "asf_internal.h"

namespace asf {
namespace {

constexpr int kLineThreads = 1024;      // setup (one workgroup, sorting)
constexpr int kLineFwdThreads = 256;    // forward (one workgroup per field)

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
        b.cell[j] = (uint32_t)c;
        for (int a = 0; a < g.w; ++a) {
            // psi at footprint cell a: z = (a - (w-1)/2 - off) 2/w
            const double z = ((double)a - 0.5 * (double)(g.w - 1) - (double)p.off) * 2.0 / (double)g.w;
            const double t = 1.0 - z * z;
            const float psi = t > 0.0 ? (float)exp(g.beta * (sqrt(t) - 1.0)) : 0.f;
            b.coef[(size_t)j * g.w + a] = make_float2(psi * p.phase.x, psi * p.phase.y);
        }
        const int cprev = j == 0 ? -1 : (int)(keys[j - 1] >> kLineKeyBits);
        for (int q = cprev + 1; q <= c; ++q) b.first[q] = (uint32_t)j;
        if (j == n - 1)
            for (int q = c + 1; q <= g.nf; ++q) b.first[q] = (uint32_t)n;
    }
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Sum over sorted points j0 <= j < j1 (their footprints start at or left of
// cell qq and cover it) of coef(j, qq - cell_j) times the field at j.
template <bool STAGED>
__device__ __forceinline__ void gather_cell(const LineBins &b, int w, const float2 *__restrict__ u,
                                            const float2 *vs, const uint32_t *cs, uint32_t j0, uint32_t j1,
                                            int qq, float &ar, float &ai) {
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t c = STAGED ? cs[j] : b.cell[j];
        const float2 k = b.coef[(size_t)j * w + (qq - (int)c)];
        const float2 v = STAGED ? vs[j] : u[b.perm[j]];
        ar = __builtin_fmaf(k.x, v.x, ar);
        ar = __builtin_fmaf(-k.y, v.y, ar);
        ai = __builtin_fmaf(k.x, v.y, ai);
        ai = __builtin_fmaf(k.y, v.x, ai);
    }
}

// STAGED: the field is first copied into LDS in sorted order (when it fits),
// so that the gather reads it there instead of through the index.
template <bool STAGED>
__global__ __launch_bounds__(kLineFwdThreads) void line_forward_kernel(LineGeo g, LineBins b,
                                                                        const float2 *__restrict__ tw,
                                                                        const float2 *__restrict__ dd,
                                                                        const float2 *__restrict__ u1,
                                                                        float2 *__restrict__ u2) {
    // nf cells, then (STAGED) the n field values, the n first cells and the nf + 1
    // run starts
    extern __shared__ float2 line[];
    const float2 *u = u1 + (size_t)blockIdx.x * g.n;
    const int nf = g.nf, w = g.w, lg = g.log_nf;
    float2 *vs = line + nf;
    uint32_t *cs = reinterpret_cast<uint32_t *>(vs + g.n);
    uint32_t *fs = cs + g.n;
    if constexpr (STAGED) {
        // four points per thread at a time: their index loads, then their gathers,
        // go out together
        constexpr int B = 4;
        for (int j0 = threadIdx.x; j0 < g.n; j0 += B * kLineFwdThreads) {
            uint32_t pj[B];
            float2 v[B];
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int j = j0 + q * kLineFwdThreads;
                pj[q] = j < g.n ? b.perm[j] : 0u;
            }
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int j = j0 + q * kLineFwdThreads;
                v[q] = j < g.n ? u[pj[q]] : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int j = j0 + q * kLineFwdThreads;
                if (j < g.n) vs[j] = v[q];
            }
        }
        for (int j = threadIdx.x; j < g.n; j += kLineFwdThreads) cs[j] = b.cell[j];
        for (int q = threadIdx.x; q <= nf; q += kLineFwdThreads) fs[q] = b.first[q];
        __syncthreads();
    }

    // spreading as a gather: the points whose footprints cover cell q are those
    // starting in cells q-w+1 .. q, one contiguous run of the sorted list (two
    // when the run wraps past cell 0)
    for (int q = threadIdx.x; q < nf; q += kLineFwdThreads) {
        float ar = 0.f, ai = 0.f;
        const int lo = q - w + 1;
        const uint32_t *first = STAGED ? fs : b.first;
        const uint32_t jq = first[q + 1];
        if (lo >= 0) {
            gather_cell<STAGED>(b, w, u, vs, cs, first[lo], jq, q, ar, ai);
        } else {
            gather_cell<STAGED>(b, w, u, vs, cs, first[lo + nf], (uint32_t)g.n, q + nf, ar, ai);
            gather_cell<STAGED>(b, w, u, vs, cs, first[0], jq, q, ar, ai);
        }
        line[__brev((unsigned)q) >> (32 - lg)] = make_float2(ar, ai);
    }
    __syncthreads();

    // in-place decimation-in-time FFT, exp(-2 pi i k q / nf), on bit-reversed input:
    // an odd number of levels starts with one radix-2 level, the rest go two at a
    // time (a radix-4 butterfly on a, a+h, a+2h, a+3h does levels h and 2h)
    int h = 1;
    if (lg & 1) {
        for (int t = threadIdx.x; t < (nf >> 1); t += kLineFwdThreads) {
            const float2 x0 = line[2 * t], x1 = line[2 * t + 1];
            line[2 * t] = make_float2(x0.x + x1.x, x0.y + x1.y);
            line[2 * t + 1] = make_float2(x0.x - x1.x, x0.y - x1.y);
        }
        __syncthreads();
        h = 2;
    }
    for (; h < nf; h <<= 2) {
        const int s2 = nf / (2 * h), s4 = nf / (4 * h);   // twiddle strides of the two levels
        for (int t = threadIdx.x; t < (nf >> 2); t += kLineFwdThreads) {
            const int pos = t & (h - 1);
            const int a = (t - pos) * 4 + pos;             // (t / h) 4h + pos
            const float2 w2 = tw[pos * s2];
            const float2 w4a = tw[pos * s4], w4b = tw[(pos + h) * s4];
            // level h: (a, a+h) and (a+2h, a+3h), twiddle w2
            const float2 p0 = line[a], p1 = cmul(line[a + h], w2);
            const float2 p2 = line[a + 2 * h], p3 = cmul(line[a + 3 * h], w2);
            const float2 q0 = make_float2(p0.x + p1.x, p0.y + p1.y), q1 = make_float2(p0.x - p1.x, p0.y - p1.y);
            const float2 q2 = make_float2(p2.x + p3.x, p2.y + p3.y), q3 = make_float2(p2.x - p3.x, p2.y - p3.y);
            // level 2h: (a, a+2h) with w4a, (a+h, a+3h) with w4b
            const float2 r2 = cmul(q2, w4a), r3 = cmul(q3, w4b);
            line[a] = make_float2(q0.x + r2.x, q0.y + r2.y);
            line[a + 2 * h] = make_float2(q0.x - r2.x, q0.y - r2.y);
            line[a + h] = make_float2(q1.x + r3.x, q1.y + r3.y);
            line[a + 3 * h] = make_float2(q1.x - r3.x, q1.y - r3.y);
        }
        __syncthreads();
    }

    // kept modes k = ix - m/2 at FFT index k mod nf, times the deconvolution and phase
    float2 *out = u2 + (size_t)blockIdx.x * g.m;
    for (int ix = threadIdx.x; ix < g.m; ix += kLineFwdThreads) {
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
    // stage the field, the first cells and the run starts in LDS when they and the
    // line together stay within 64 KB
    const size_t line_bytes = sizeof(float2) * (size_t)g.nf;
    const size_t staged_bytes = line_bytes + (sizeof(float2) + sizeof(uint32_t)) * (size_t)g.n +
                                sizeof(uint32_t) * ((size_t)g.nf + 1);
    if (staged_bytes <= 65536) {
        hipLaunchKernelGGL(line_forward_kernel<true>, dim3(batch), dim3(kLineFwdThreads), staged_bytes, s,
                           g, b, tw, dd, u1, u2);
        return hipGetLastError();
    }
    static size_t enabled = 0;
    if (line_bytes > 65536 && line_bytes > enabled) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(line_forward_kernel<false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)line_bytes);
        if (e != hipSuccess) return e;
        enabled = line_bytes;
    }
    hipLaunchKernelGGL(line_forward_kernel<false>, dim3(batch), dim3(kLineFwdThreads), line_bytes, s,
                       g, b, tw, dd, u1, u2);
    return hipGetLastError();
}

}  // namespace asf
