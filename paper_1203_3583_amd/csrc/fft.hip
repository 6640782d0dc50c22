// Uniform FFT on gfx950: the "uniform FFT" half of the non-uniform FFT the
// paper evaluates Eq. (9) with (Sec. 2), plus the deconvolution, crop and
// destination phase of Eq. (8) fused into the last pass.
//
// A 2D forward DFT (exp(-i) sign) of the nfx x nfy fine grid is done in two
// passes, each pruned to the modes the destination grid keeps:
//   pass 1: every fine-grid column (length nfy), keep the my centred modes,
//           write mid[ky][lx] (my x nfx, row-major);
//   pass 2: every mid row (length nfx), keep the mx centred modes, multiply by
//           Dx[ix] Dy[iy] (1/psi-hat, the destination chirp of Eq. (6)/(7) and
//           the prefactor exp(i k z0)/(i lambda z0)) and write u2[iy][ix].
// A workgroup holds `batch` whole transforms in LDS.  Each transform of length
// L = r0 * 16^a runs as Stockham stages: one radix-r0 stage (r0 in {1,2,4,8})
// on the vector ALU, then a radix-16 stages.  In a radix-16 stage the 16-point
// DFTs of 16 transform instances form one small GEMM
//     [Re Y; Im Y] (32 x 16) = W16 (32 x 32 real form of the DFT matrix) x [Re X; Im X] (32 x 16)
// run on the matrix cores, either with FP32 products (v_mfma_f32_16x16x4_f32,
// 8 K-steps per output half) or with FP16 hi+lo split products
// (v_mfma_f32_16x16x32_f16: W_hi X_hi + W_hi X_lo + W_lo X_hi with FP32
// accumulation, X scaled per instance by a power of two so the split stays in
// FP16 range).  Twiddles are applied in FP32 on the vector ALU before each
// stage's DFT, from an FP64-computed table.
//
// Lane layout of one 16-instance block (wave64): lane = 16 g + jj holds instance
// jj's inputs r = g, g+4, g+8, g+12 and, after the MFMAs, its outputs
// p = g, g+4, g+8, g+12 (the DFT matrix rows are permuted so that the 16 x 16
// accumulator's rows 4g..4g+3 are those outputs).  The K index of both operands
// is permuted the same way, (r, re/im) <-> K slot, which the MFMA contraction
// does not see.
#include "asf_internal.h"

namespace asf {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS position of element e of a transform: the low 4 bits are XOR-swizzled by
// bits 4..7 and 16 slots of padding follow every 2^pad_shift elements, which
// keeps the stage reads and writes of a half-wave on distinct banks.
__device__ inline int lds_pos(int e, int pad_shift) {
    return (e ^ ((e >> 4) & 15)) + ((e >> pad_shift) << 4);
}

struct Stage {
    int L, r0, n16, lq, lq_shift, batch, stride, pad_shift;
};

// A-operand (DFT matrix) fragments for this lane, built from w16[q] = exp(-2 pi i q / 16).
struct Dft16F32 {
    float are[8], aim[8];
    __device__ void init(const float2 *w16, int g, int jj) {
        const int p = (jj >> 2) + 4 * (jj & 3);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            const int r = g + 4 * (kb >> 1);
            const float2 w = w16[(p * r) & 15];
            are[kb] = (kb & 1) ? -w.y : w.x;
            aim[kb] = (kb & 1) ? w.x : w.y;
        }
    }
    __device__ void run(float2 (&v)[4]) const {
        v4f accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            const float b = (kb & 1) ? v[kb >> 1].y : v[kb >> 1].x;
            accr = __builtin_amdgcn_mfma_f32_16x16x4f32(are[kb], b, accr, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[kb], b, acci, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = make_float2(accr[i], acci[i]);
    }
};

struct Dft16Split16 {
    v8h re_hi, re_lo, im_hi, im_lo;
    __device__ void init(const float2 *w16, int g, int jj) {
        const int p = (jj >> 2) + 4 * (jj & 3);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int r = g + 4 * (e >> 1);
            const float2 w = w16[(p * r) & 15];
            const float a = (e & 1) ? -w.y : w.x;
            const float b = (e & 1) ? w.x : w.y;
            const _Float16 ah = (_Float16)a, bh = (_Float16)b;
            re_hi[e] = ah;
            re_lo[e] = (_Float16)(a - (float)ah);
            im_hi[e] = bh;
            im_lo[e] = (_Float16)(b - (float)bh);
        }
    }
    __device__ void run(float2 (&v)[4]) const {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) m = fmaxf(m, fmaxf(fabsf(v[i].x), fabsf(v[i].y)));
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        int ex = 0;
        if (m > 0.f) frexpf(m, &ex);
        const float inv = ldexpf(1.f, -ex), sc = ldexpf(1.f, ex);
        v8h bh, bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float val = ((e & 1) ? v[e >> 1].y : v[e >> 1].x) * inv;
            const _Float16 h = (_Float16)val;
            bh[e] = h;
            bl[e] = (_Float16)(val - (float)h);
        }
        v4f accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_lo, bh, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_lo, bh, acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_hi, bl, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_hi, bl, acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_hi, bh, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_hi, bh, acci, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = make_float2(accr[i] * sc, acci[i] * sc);
    }
};

// Radix-R0 first stage (Ns = 1, no twiddles) on the vector ALU, in place.
template <int R0, int BPW>
__device__ void first_stage(float2 *lds, const Stage &st, const float2 *w16s) {
    if constexpr (R0 > 1) {
        constexpr int IPT = (4 * BPW) / R0 > 0 ? (4 * BPW) / R0 : 1;  // instances per thread
        const int nt = blockDim.x;
        const int per = st.L / R0;
        const int ninst = st.batch * per;
        float2 v[IPT][R0];
#pragma unroll
        for (int a = 0; a < IPT; ++a) {
            const int inst = threadIdx.x + a * nt;
            if (inst < ninst) {
                const int c = inst / per, j = inst - c * per;
                float2 x[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) x[r] = lds[c * st.stride + lds_pos(j + r * per, st.pad_shift)];
#pragma unroll
                for (int p = 0; p < R0; ++p) {
                    float2 acc = x[0];
#pragma unroll
                    for (int r = 1; r < R0; ++r) {
                        const float2 w = w16s[(p * r * (16 / R0)) & 15];
                        acc.x += x[r].x * w.x - x[r].y * w.y;
                        acc.y += x[r].x * w.y + x[r].y * w.x;
                    }
                    v[a][p] = acc;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < IPT; ++a) {
            const int inst = threadIdx.x + a * nt;
            if (inst < ninst) {
                const int c = inst / per, j = inst - c * per;
#pragma unroll
                for (int p = 0; p < R0; ++p) lds[c * st.stride + lds_pos(j * R0 + p, st.pad_shift)] = v[a][p];
            }
        }
        __syncthreads();
    }
}

// All radix-16 stages, in place in LDS.
template <class Engine, int R0, int BPW>
__device__ void radix16_stages(float2 *lds, const Stage &st, const float2 *__restrict__ tw,
                               const Engine &eng) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jj = lane & 15;
    const int wave = threadIdx.x >> 6;
    const int lq = st.lq;
    int ns = R0;
    for (int s = 0; s < st.n16; ++s) {
        float2 v[BPW][4];
        const int tstep = lq / ns;   // twiddle index step: L / (16 ns)
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int q = (wave * BPW + b) * 16 + jj;
            const int c = q >> st.lq_shift, j = q & (lq - 1);
            const int k = j & (ns - 1);
            const float2 *col = lds + c * st.stride;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = g + 4 * i;
                float2 x = col[lds_pos(j + r * lq, st.pad_shift)];
                if (ns > 1) x = cmul(x, tw[r * k * tstep]);
                v[b][i] = x;
            }
            eng.run(v[b]);
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int q = (wave * BPW + b) * 16 + jj;
            const int c = q >> st.lq_shift, j = q & (lq - 1);
            const int k = j & (ns - 1);
            const int base = (j - k) * 16 + k;   // (j / ns) * 16 ns + k
            float2 *col = lds + c * st.stride;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = g + 4 * i;
                col[lds_pos(base + p * ns, st.pad_shift)] = v[b][i];
            }
        }
        __syncthreads();
        ns *= 16;
    }
}

template <int SPLIT, int R0, int BPW>
__device__ void transform_all(float2 *lds, const Stage &st, const float2 *tw, const float2 *w16) {
    __shared__ float2 w16s[16];
    if (threadIdx.x < 16) w16s[threadIdx.x] = w16[threadIdx.x];
    __syncthreads();
    first_stage<R0, BPW>(lds, st, w16s);
    const int lane = threadIdx.x & 63;
    if constexpr (SPLIT) {
        Dft16Split16 eng;
        eng.init(w16s, lane >> 4, lane & 15);
        radix16_stages<Dft16Split16, R0, BPW>(lds, st, tw, eng);
    } else {
        Dft16F32 eng;
        eng.init(w16s, lane >> 4, lane & 15);
        radix16_stages<Dft16F32, R0, BPW>(lds, st, tw, eng);
    }
}

// Pass 1: workgroup = one panel of `batch` adjacent fine-grid columns.
template <int SPLIT, int R0, int BPW>
__global__ void __launch_bounds__(1024) fft_pass1_kernel(Stage st, const float2 *__restrict__ fine,
                                                         float2 *__restrict__ mid,
                                                         const float2 *__restrict__ tw,
                                                         const float2 *__restrict__ w16, int nfx,
                                                         int my) {
    extern __shared__ float2 lds[];
    const int C = st.batch, L = st.L;
    const int pc = blockIdx.x;
    const float2 *src = fine + (size_t)pc * L * C;
    for (int t = threadIdx.x; t < L * C; t += blockDim.x) {
        const int ly = t / C, c = t - ly * C;
        lds[c * st.stride + lds_pos(ly, st.pad_shift)] = src[t];
    }
    __syncthreads();
    transform_all<SPLIT, R0, BPW>(lds, st, tw, w16);
    const int half = my >> 1;
    for (int t = threadIdx.x; t < my * C; t += blockDim.x) {
        const int ky = t / C, c = t - ky * C;
        int l = ky - half;
        if (l < 0) l += L;
        mid[(size_t)ky * nfx + pc * C + c] = lds[c * st.stride + lds_pos(l, st.pad_shift)];
    }
}

// Pass 2: workgroup = `batch` rows of mid; fused deconvolution and phase.
template <int SPLIT, int R0, int BPW>
__global__ void __launch_bounds__(1024) fft_pass2_kernel(Stage st, const float2 *__restrict__ mid,
                                                         float2 *__restrict__ u2,
                                                         const float2 *__restrict__ tw,
                                                         const float2 *__restrict__ w16,
                                                         const float2 *__restrict__ dx,
                                                         const float2 *__restrict__ dy, int mx) {
    extern __shared__ float2 lds[];
    const int C = st.batch, L = st.L;
    const int row0 = blockIdx.x * C;
    const float2 *src = mid + (size_t)row0 * L;
    for (int t = threadIdx.x; t < L * C; t += blockDim.x) {
        const int c = t / L, lx = t - c * L;
        lds[c * st.stride + lds_pos(lx, st.pad_shift)] = src[t];
    }
    __syncthreads();
    transform_all<SPLIT, R0, BPW>(lds, st, tw, w16);
    const int half = mx >> 1;
    for (int t = threadIdx.x; t < mx * C; t += blockDim.x) {
        const int c = t / mx, ix = t - c * mx;
        int l = ix - half;
        if (l < 0) l += L;
        const float2 val = lds[c * st.stride + lds_pos(l, st.pad_shift)];
        u2[(size_t)(row0 + c) * mx + ix] = cmul(cmul(val, dx[ix]), dy[row0 + c]);
    }
}

Stage make_stage(const FftShape &sh) {
    Stage st;
    st.L = sh.L;
    st.r0 = sh.r0;
    st.n16 = sh.n16;
    st.lq = sh.lq;
    int s = 0;
    while ((1 << s) < sh.lq) ++s;
    st.lq_shift = s;
    st.batch = sh.batch;
    st.stride = sh.stride;
    int ps = 0;
    const int unit = sh.lq > 16 ? sh.lq : 16;
    while ((1 << ps) < unit) ++ps;
    st.pad_shift = ps;
    return st;
}

// Kernels needing more than 64 KB of dynamic LDS must say so once per size.
hipError_t allow_lds(const void *kernel, size_t lds, size_t &enabled) {
    if (lds > 65536 && lds > enabled) {
        hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        enabled = lds;
    }
    return hipSuccess;
}

template <int PASS, int SPLIT, int R0, int BPW>
hipError_t launch_t(const FftShape &sh, const float2 *in, float2 *out, const float2 *tw,
                    const float2 *w16, const float2 *dx, const float2 *dy, int nx_out, int n_other,
                    hipStream_t s) {
    const Stage st = make_stage(sh);
    const size_t lds = fft_lds_bytes(sh);
    const dim3 block(64 * sh.waves);
    static thread_local size_t enabled = 0;   // per instantiation and host thread
    if (PASS == 1) {
        auto k = fft_pass1_kernel<SPLIT, R0, BPW>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        const int groups = nx_out / sh.batch;   // nfx / batch panels
        hipLaunchKernelGGL(k, dim3(groups), block, lds, s, st, in, out, tw, w16, nx_out, n_other);
    } else {
        auto k = fft_pass2_kernel<SPLIT, R0, BPW>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        const int groups = n_other / sh.batch;  // my / batch row groups
        hipLaunchKernelGGL(k, dim3(groups), block, lds, s, st, in, out, tw, w16, dx, dy, nx_out);
    }
    return hipGetLastError();
}

template <int PASS, int SPLIT, int R0>
hipError_t launch_bpw(const FftShape &sh, const float2 *in, float2 *out, const float2 *tw,
                      const float2 *w16, const float2 *dx, const float2 *dy, int nx_out,
                      int n_other, hipStream_t s) {
    switch (sh.bpw) {
        case 1: return launch_t<PASS, SPLIT, R0, 1>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        case 2: return launch_t<PASS, SPLIT, R0, 2>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        case 4: return launch_t<PASS, SPLIT, R0, 4>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PASS, int SPLIT>
hipError_t launch_r0(const FftShape &sh, const float2 *in, float2 *out, const float2 *tw,
                     const float2 *w16, const float2 *dx, const float2 *dy, int nx_out, int n_other,
                     hipStream_t s) {
    switch (sh.r0) {
        case 1: return launch_bpw<PASS, SPLIT, 1>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        case 2: return launch_bpw<PASS, SPLIT, 2>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        case 4: return launch_bpw<PASS, SPLIT, 4>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        case 8: return launch_bpw<PASS, SPLIT, 8>(sh, in, out, tw, w16, dx, dy, nx_out, n_other, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t fft_lds_bytes(const FftShape &sh) { return (size_t)sh.batch * sh.stride * sizeof(float2); }

int fft_max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

hipError_t launch_fft_pass1(const FftShape &sh, int split16, const float2 *fine, float2 *mid,
                            const float2 *tw, const float2 *w16, int nfx, int my, hipStream_t s) {
    if (split16) return launch_r0<1, 1>(sh, fine, mid, tw, w16, nullptr, nullptr, nfx, my, s);
    return launch_r0<1, 0>(sh, fine, mid, tw, w16, nullptr, nullptr, nfx, my, s);
}

hipError_t launch_fft_pass2(const FftShape &sh, int split16, const float2 *mid, float2 *u2,
                            const float2 *tw, const float2 *w16, const float2 *dx,
                            const float2 *dy, int mx, int my, hipStream_t s) {
    if (split16) return launch_r0<2, 1>(sh, mid, u2, tw, w16, dx, dy, mx, my, s);
    return launch_r0<2, 0>(sh, mid, u2, tw, w16, dx, dy, mx, my, s);
}

}  // namespace asf
