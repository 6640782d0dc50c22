// Uniform FFT on gfx950: the "uniform FFT" half of the non-uniform FFT the
// paper evaluates Eq. (9) with (Sec. 2), plus the deconvolution, crop and
// destination phase of Eq. (8) fused into the last pass.
//
// A 2D forward DFT (exp(-i) sign) of the nfx x nfy fine grid is done in two
// passes, each pruned to the modes the destination grid keeps:
//   pass 1: every fine-grid column (length nfy; where the plan leaves the tiles no
//           record reaches unwritten, their cells read as zeros without a load, and
//           a panel of columns with no such tile writes zeros without a transform),
//           keep the my centred modes,
//           write them to mid in the fine grid's panel layout (panels of C
//           adjacent columns, element (lx, ky) at ((lx / C) my + ky) C + lx % C),
//           so that each workgroup writes one contiguous block;
//   pass 2: every mid row (length nfx), gathered from the panels (C elements at
//           a time; the 16 / C rows that share a 128-byte line run on one XCD,
//           whose L2 serves the line to all of them), keep the mx centred
//           modes, multiply by
//           Dx[ix] Dy[iy] (1/psi-hat, the destination chirp of Eq. (6)/(7) and
//           the prefactor exp(i k z0)/(i lambda z0)) and write u2[iy][ix].
// A workgroup holds `batch` whole transforms in LDS.  Each transform of length
// L = r0 * 16^a (a compile-time constant here, so every index is a shift or a
// constant offset) runs as Stockham stages: one radix-r0 stage (r0 in
// {1,2,4,8}) on the vector ALU, then a radix-16 stages, each a 16-point DFT of
// 16 transform instances per wave and block, in one of two engines:
//   FP32 (vector ALU): 4 x 4 -- a 4-point DFT over the four inputs a lane
//     holds, twiddles W16^(g k1), a transpose of the block's four 16-lane rows
//     by lane swaps, a second 4-point DFT (about 50 operations per lane);
//   split FP16 (matrix cores): the 16-point DFT as one small GEMM
//     [Re Y; Im Y] (32 x 16) = W16 (32 x 32 real form of the DFT matrix) x [Re X; Im X] (32 x 16)
//     with FP16 hi+lo split products (v_mfma_f32_16x16x32_f16: W_hi X_hi +
//     W_hi X_lo + W_lo X_hi, FP32 accumulation).  The workgroup scales its data
//     once, at load, by a power of two that brings the largest |Re|, |Im| to at
//     most 1: FP16 carries its own exponent, so the scale only guards the
//     range, and a transform of length L grows values by at most L <= 16384 <
//     65504.
// On gfx950 the FP32 matrix rate equals the FP32 vector rate, and a dense
// 16-point DFT costs about six times the operations of the 4 x 4 network, so
// FP32 products stay on the vector ALU.
// Twiddles are applied in FP32 on the vector ALU before each stage's DFT, from
// FP64-computed tables laid out [k][lane group][4] so that a lane fetches its
// four twiddles with two 16-byte loads.
//
// Lane layout of one 16-instance block (wave64): lane = 16 g + jj holds instance
// jj's inputs r = g, g+4, g+8, g+12 and, after the DFT, its outputs
// p = g, g+4, g+8, g+12 (for the GEMM the DFT matrix rows are permuted so that
// the 16 x 16 accumulator's rows 4g..4g+3 are those outputs, and the K index of
// both operands is permuted the same way, (r, re/im) <-> K slot, which the
// contraction does not see).
#include <type_traits>

#include "asf_internal.h"

namespace asf {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Compile-time shape of one transform length.
template <int LOGL>
struct Len {
    static constexpr int L = 1 << LOGL;
    static constexpr int N16 = LOGL / 4;          // radix-16 stages
    static constexpr int R0 = 1 << (LOGL % 4);    // first (vector ALU) radix
    static constexpr int LQ = L / 16;
    static constexpr int LOGLQ = LOGL - 4;
    static constexpr int PS = LQ > 16 ? LOGLQ : 4;            // one pad of 16 per 2^PS elements
    static constexpr int STRIDE = L + (L >> PS) * 16;          // LDS elements per transform
};

// LDS position of element e: low 4 bits XOR-swizzled by bits 4..7, plus 16 slots
// of padding every 2^PS elements (keeps a half-wave's accesses on distinct banks).
template <int PS>
__device__ __forceinline__ int lds_pos(int e) {
    return (e ^ ((e >> 4) & 15)) + ((e >> PS) << 4);
}

// 16-point DFTs on the vector ALU in FP32, as 4 x 4 (r = g + 4 i,
// p = k1 + 4 k2):
//   Y[k1 + 4 k2] = sum_g W4^(g k2) W16^(g k1) sum_i x[g + 4 i] W4^(i k1).
// A lane holds x[g + 4 i] for i = 0..3, so the inner 4-point DFT and the twiddle
// W16^(g k1) (g is the lane's row of 16 lanes) stay in its registers; a 4 x 4
// transpose of (row, register) -- two v_permlane32_swap and two
// v_permlane16_swap per real component -- gives row k1 the values of all four
// g, and the outer 4-point DFT leaves Y[g + 4 k2] in register k2 of row g: the
// layout the matrix-core engine produces.  About 50 VALU operations per lane and
// block, where the same DFT as a GEMM takes 16 FP32 MFMAs of 32 cycles.
struct Dft16Valu {
    float2 w1, w2, w3;   // W16^g, W16^2g, W16^3g for this lane's row g
    __device__ __forceinline__ void init(const float2 *w16, int g, int) {
        w1 = w16[g & 15];
        w2 = w16[(2 * g) & 15];
        w3 = w16[(3 * g) & 15];
    }
    // forward 4-point DFT (W4 = -i) in place
    static __device__ __forceinline__ void dft4(float2 (&v)[4]) {
        const float2 a0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 a1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 a2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 a3 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        v[0] = make_float2(a0.x + a2.x, a0.y + a2.y);
        v[2] = make_float2(a0.x - a2.x, a0.y - a2.y);
        v[1] = make_float2(a1.x + a3.y, a1.y - a3.x);   // a1 - i a3
        v[3] = make_float2(a1.x - a3.y, a1.y + a3.x);   // a1 + i a3
    }
    // (row, register) transpose of one real component over the wave's four rows
    static __device__ __forceinline__ void transpose4(float &r0, float &r1, float &r2, float &r3) {
        auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r0), __float_as_uint(r2), false, false);
        auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r1), __float_as_uint(r3), false, false);
        auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
        auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
        r0 = __uint_as_float(s01[0]);
        r1 = __uint_as_float(s01[1]);
        r2 = __uint_as_float(s23[0]);
        r3 = __uint_as_float(s23[1]);
    }
    __device__ __forceinline__ void run(float2 (&v)[4]) const {
        dft4(v);
        v[1] = cmul(v[1], w1);
        v[2] = cmul(v[2], w2);
        v[3] = cmul(v[3], w3);
        transpose4(v[0].x, v[1].x, v[2].x, v[3].x);
        transpose4(v[0].y, v[1].y, v[2].y, v[3].y);
        dft4(v);
    }
};

struct Dft16Split16 {
    v8h re_hi, re_lo, im_hi, im_lo;
    __device__ __forceinline__ void init(const float2 *w16, int g, int jj) {
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
    // inputs already scaled into FP16 range by the workgroup's scale
    __device__ __forceinline__ void run(float2 (&v)[4]) const {
        v8h bh, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const v2f x = {v[i].x, v[i].y};
            const v2h h = __builtin_convertvector(x, v2h);
            const v2f r = x - __builtin_convertvector(h, v2f);
            const v2h l = __builtin_convertvector(r, v2h);
            bh[2 * i] = h.x;
            bh[2 * i + 1] = h.y;
            bl[2 * i] = l.x;
            bl[2 * i + 1] = l.y;
        }
        v4f accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_lo, bh, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_lo, bh, acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_hi, bl, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_hi, bl, acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re_hi, bh, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_f16(im_hi, bh, acci, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = make_float2(accr[i], acci[i]);
    }
};

// Radix-R0 first stage (Ns = 1, no twiddles) on the vector ALU, in place.
template <int LOGL, int BATCH, int NT, bool SCALE>
__device__ __forceinline__ void first_stage(float2 *lds, const float2 *w16s, float inv) {
    using S = Len<LOGL>;
    constexpr int R0 = S::R0;
    if constexpr (R0 > 1) {
        constexpr int PER = S::L / R0;
        constexpr int NINST = BATCH * PER;
        constexpr int IPT = (NINST + NT - 1) / NT;
        float2 v[IPT][R0];
#pragma unroll
        for (int a = 0; a < IPT; ++a) {
            const int inst = threadIdx.x + a * NT;
            if (inst < NINST) {
                const int c = inst / PER, j = inst % PER;
                float2 x[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    x[r] = lds[c * S::STRIDE + lds_pos<S::PS>(j + r * PER)];
                    if constexpr (SCALE) x[r] = make_float2(x[r].x * inv, x[r].y * inv);
                }
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
            const int inst = threadIdx.x + a * NT;
            if (inst < NINST) {
                const int c = inst / PER, j = inst % PER;
#pragma unroll
                for (int p = 0; p < R0; ++p) lds[c * S::STRIDE + lds_pos<S::PS>(j * R0 + p)] = v[a][p];
            }
        }
        __syncthreads();
    }
}

// 16-instance blocks of a radix-16 stage per wave
template <int LOGL, int BATCH, int NT>
struct StageBlocks {
    static constexpr int BLOCKS = BATCH * Len<LOGL>::LQ / 16;
    static constexpr int WAVES = NT / 64;
    static constexpr int BPW = BLOCKS / WAVES;
    static_assert(BLOCKS % WAVES == 0 && BPW >= 1, "blocks must divide among waves");
};

// This lane's twiddles of a stage with span NS (table entry (k, g, i) =
// exp(-2 pi i (g + 4 i) k / (16 NS))): two 16-byte loads per block.  A stage's
// twiddles are fetched during the previous stage, before its last barrier, so
// that their latency hides behind the barrier instead of stalling the stage.
template <int LOGL, int BATCH, int NT, int NS>
__device__ __forceinline__ void load_twiddles(const float4 *__restrict__ tw,
                                              float4 (&t)[StageBlocks<LOGL, BATCH, NT>::BPW][2]) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    if constexpr (NS > 1) {
        const int lane = threadIdx.x & 63;
        const int g = lane >> 4, jj = lane & 15, wave = threadIdx.x >> 6;
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int j = ((wave * BPW + b) * 16 + jj) & (S::LQ - 1);
            const float4 *p = tw + ((j & (NS - 1)) * 16 + g * 4) / 2;
            t[b][0] = p[0];
            t[b][1] = p[1];
        }
    }
}

// One radix-16 Stockham stage with span NS, in place in LDS, with this stage's
// twiddles already in registers (tcur); fetches the next stage's (span NSN,
// table twn) into tnext.
template <int LOGL, int BATCH, int NT, int NS, int NSN, bool SCALE, class Engine>
__device__ __forceinline__ void radix16_stage(
    float2 *lds, const float4 (&tcur)[StageBlocks<LOGL, BATCH, NT>::BPW][2], const float4 *__restrict__ twn,
    float4 (&tnext)[StageBlocks<LOGL, BATCH, NT>::BPW][2], const Engine &eng, float inv) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jj = lane & 15;
    const int wave = threadIdx.x >> 6;
    float2 v[BPW][4];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int q = (wave * BPW + b) * 16 + jj;
        const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
        const float2 *col = lds + c * S::STRIDE;
        if constexpr (S::LQ >= 64) {
            // e + 4 i LQ changes neither bits 4..7 of e nor e mod 2^PS: the swizzled
            // positions of the four inputs are one base plus constant offsets
            const float2 *src = col + lds_pos<S::PS>(j + g * S::LQ);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = src[i * (4 * S::LQ + 64)];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = col[lds_pos<S::PS>(j + (g + 4 * i) * S::LQ)];
        }
        if constexpr (SCALE) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = make_float2(v[b][i].x * inv, v[b][i].y * inv);
        }
        if constexpr (NS > 1) {
            const float4 t01 = tcur[b][0], t23 = tcur[b][1];
            v[b][0] = cmul(v[b][0], make_float2(t01.x, t01.y));
            v[b][1] = cmul(v[b][1], make_float2(t01.z, t01.w));
            v[b][2] = cmul(v[b][2], make_float2(t23.x, t23.y));
            v[b][3] = cmul(v[b][3], make_float2(t23.z, t23.w));
        }
        eng.run(v[b]);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int q = (wave * BPW + b) * 16 + jj;
        const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
        const int k = j & (NS - 1);
        const int base = (j - k) * 16 + k;   // (j / NS) * 16 NS + k
        float2 *col = lds + c * S::STRIDE;
        if constexpr (NS >= 64 && (4 * NS) % S::LQ == 0) {
            // as for the reads: 4 i NS is a multiple of 256 and of 2^PS
            float2 *dst = col + lds_pos<S::PS>(base + g * NS);
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[i * (4 * NS + ((4 * NS) >> S::PS) * 16)] = v[b][i];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) col[lds_pos<S::PS>(base + (g + 4 * i) * NS)] = v[b][i];
        }
    }
    load_twiddles<LOGL, BATCH, NT, NSN>(twn, tnext);
    __syncthreads();
}

// Offset (in complex entries) of stage STAGE's twiddle table: tables are stored
// only for stages with span NS > 1, in stage order, 16 NS entries each.
template <int LOGL>
constexpr int twiddle_offset(int stage) {
    int off = 0;
    for (int s = 0; s < stage; ++s) {
        const int ns = Len<LOGL>::R0 << (4 * s);
        if (ns > 1) off += 16 * ns;
    }
    return off;
}

template <int LOGL>
__device__ __forceinline__ const float4 *stage_table(const float4 *tw, int stage) {
    return reinterpret_cast<const float4 *>(reinterpret_cast<const float2 *>(tw) + twiddle_offset<LOGL>(stage));
}

// SCALE: multiply the transform's input by inv as the first stage reads it
template <int LOGL, int BATCH, int NT, int STAGE, bool SCALE, class Engine>
__device__ __forceinline__ void stages_from(float2 *lds, const float4 *tw, const Engine &eng,
                                            const float4 (&tcur)[StageBlocks<LOGL, BATCH, NT>::BPW][2],
                                            float inv) {
    using S = Len<LOGL>;
    if constexpr (STAGE < S::N16) {
        constexpr int NS = S::R0 << (4 * STAGE);
        constexpr int NSN = STAGE + 1 < S::N16 ? NS * 16 : 1;   // 1: no next stage to fetch for
        constexpr bool SC = SCALE && STAGE == 0 && S::R0 == 1;   // else first_stage scaled
        float4 tnext[StageBlocks<LOGL, BATCH, NT>::BPW][2];
        radix16_stage<LOGL, BATCH, NT, NS, NSN, SC, Engine>(lds, tcur, stage_table<LOGL>(tw, STAGE + 1), tnext,
                                                            eng, inv);
        stages_from<LOGL, BATCH, NT, STAGE + 1, SCALE, Engine>(lds, tw, eng, tnext, inv);
    }
}

// The workgroup's transforms, in place in LDS; with SPLIT the input is scaled by
// inv (a power of two) on its way into the first stage.
template <int LOGL, int BATCH, int NT, bool SPLIT>
__device__ __forceinline__ void transform_all(float2 *lds, const float2 *tw, const float2 *w16, float inv) {
    __shared__ float2 w16s[16];
    const float4 *tw4 = reinterpret_cast<const float4 *>(tw);
    float4 t0[StageBlocks<LOGL, BATCH, NT>::BPW][2];
    load_twiddles<LOGL, BATCH, NT, Len<LOGL>::R0>(stage_table<LOGL>(tw4, 0), t0);   // first radix-16 stage
    if (threadIdx.x < 16) w16s[threadIdx.x] = w16[threadIdx.x];
    __syncthreads();
    first_stage<LOGL, BATCH, NT, SPLIT>(lds, w16s, inv);
    const int lane = threadIdx.x & 63;
    if constexpr (SPLIT) {
        Dft16Split16 eng;
        eng.init(w16s, lane >> 4, lane & 15);
        stages_from<LOGL, BATCH, NT, 0, true, Dft16Split16>(lds, tw4, eng, t0, inv);
    } else {
        Dft16Valu eng;
        eng.init(w16s, lane >> 4, lane & 15);
        stages_from<LOGL, BATCH, NT, 0, false, Dft16Valu>(lds, tw4, eng, t0, inv);
    }
}

__device__ __forceinline__ float block_max(float v, float *scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmaxf(s, scratch[i]);
    return s;
}

// power of two 2^e with max_abs * 2^-e <= 1 (1 for zero data)
__device__ __forceinline__ int range_exponent(float max_abs) {
    int e = 0;
    if (max_abs > 0.f) frexpf(max_abs, &e);
    return e;
}

// With flags (tiles no record reaches, left unwritten): the flags of the tile column
// holding fine-grid column x0, one byte per tile row, into LDS.  Returns whether
// flags are in use.
__device__ __forceinline__ bool live_rows(const LiveTiles &lt, int x0, uint8_t *lrow) {
    if (!lt.flag) return false;
    const uint8_t *col = lt.flag + (x0 >> lt.log_tile_x);
    for (int i = threadIdx.x; i < lt.nty; i += blockDim.x) lrow[i] = col[(size_t)i * lt.ntx];
    __syncthreads();
    return true;
}

// With flags: whether the tile column holding fine-grid column x0 has a flagged tile
// (the same answer in every thread).  The columns of one with none are zeros: the
// column passes skip them, and the row passes neither read nor write them in mid.
__device__ __forceinline__ bool column_needed(const LiveTiles &lt, int x0) {
    return !lt.flag || lt.col[x0 >> lt.log_tile_x] != 0;
}

// With flags: the tile columns' flags, one byte per tile column, into LDS.  Returns
// whether flags are in use.
__device__ __forceinline__ bool live_cols(const LiveTiles &lt, uint8_t *lcol) {
    if (!lt.flag) return false;
    for (int i = threadIdx.x; i < lt.ntx; i += blockDim.x) lcol[i] = lt.col[i];
    __syncthreads();
    return true;
}

// Pass 1: a workgroup transforms one panel of BATCH adjacent fine-grid columns
// (mid's panels hold MP >= BATCH columns, as in the direct-I/O kernel below).
template <int LOGL, int BATCH, int NT, bool SPLIT, int MP>
__global__ void __launch_bounds__(NT) fft_pass1_kernel(const float2 *__restrict__ fine,
                                                       float2 *__restrict__ mid,
                                                       const float2 *__restrict__ tw,
                                                       const float2 *__restrict__ w16, int my,
                                                       LiveTiles lt, int xcd_pair) {
    using S = Len<LOGL>;
    static_assert(MP % BATCH == 0, "mid panels hold whole column batches");
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lrow[kMaxTileRows];
    int pc = blockIdx.x;
    if (MP > BATCH && xcd_pair) {
        constexpr int G = MP / BATCH;
        const int xcd = pc & 7, slot = pc >> 3;
        pc = ((slot / G) * 8 + xcd) * G + slot % G;
    }
    const float2 *src = fine + (size_t)pc * S::L * BATCH;
    if (!column_needed(lt, pc * BATCH)) return;
    const bool sparse = live_rows(lt, pc * BATCH, lrow);
    float big = 0.f;
    // every load in flight before the first LDS write (none for tiles left unwritten)
    constexpr int PER = S::L * BATCH / NT;
    float2 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        v[k] = (!sparse || lrow[(t / BATCH) >> lt.log_tile_y]) ? src[t] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int ly = t / BATCH, c = t % BATCH;
        lds[c * S::STRIDE + lds_pos<S::PS>(ly)] = v[k];
        if constexpr (SPLIT) big = fmaxf(big, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    }
    // split products: scale the workgroup's data by a power of two into FP16 range
    // (applied as the first stage reads it); the block maximum's barrier also
    // completes the LDS writes above, as transform_all's first barrier does otherwise
    float unscale = 1.f, inv = 1.f;
    if constexpr (SPLIT) {
        const int e = range_exponent(block_max(big, scratch));
        inv = ldexpf(1.f, -e);
        unscale = ldexpf(1.f, e);
    }
    transform_all<LOGL, BATCH, NT, SPLIT>(lds, tw, w16, inv);
    const int half = my >> 1;
    const int x0 = pc * BATCH;
    float2 *dst = mid + (size_t)(x0 / MP) * my * MP + x0 % MP;   // this batch's columns of its mid panel
    for (int t = threadIdx.x; t < my * BATCH; t += NT) {
        const int ky = t / BATCH, c = t % BATCH;
        const int l = (ky - half) & (S::L - 1);
        const float2 v = lds[c * S::STRIDE + lds_pos<S::PS>(l)];
        dst[ky * MP + c] = make_float2(v.x * unscale, v.y * unscale);
    }
}

// Pass 2: a workgroup transforms BATCH rows of mid; fused deconvolution and phase.
template <int LOGL, int BATCH, int NT, bool SPLIT>
__global__ void __launch_bounds__(NT) fft_pass2_kernel(const float2 *__restrict__ mid,
                                                       float2 *__restrict__ u2,
                                                       const float2 *__restrict__ tw,
                                                       const float2 *__restrict__ w16,
                                                       const float2 *__restrict__ dx,
                                                       const float2 *__restrict__ dy, int mx,
                                                       int my, int log_panel, int xcd_group,
                                                       int accumulate, LiveTiles lt) {
    using S = Len<LOGL>;
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lcol[kMaxTileCols];
    // workgroups are dealt to the 8 XCDs round-robin: give the xcd_group
    // workgroups whose rows share lines of mid consecutive slots on one XCD
    int g = blockIdx.x;
    if (xcd_group > 1) {
        const int xcd = g & 7, slot = g >> 3;
        g = ((slot / xcd_group) * 8 + xcd) * xcd_group + slot % xcd_group;
    }
    const int row0 = g * BATCH;
    const int cmask = (1 << log_panel) - 1;
    const bool sparse = live_cols(lt, lcol);
    float big = 0.f;
    // every load in flight before the first LDS write (a row is gathered from
    // the panels, one line per element: serial round trips would dominate);
    // columns the column pass skipped are zeros, not loaded
    constexpr int PER = S::L * BATCH / NT;
    float2 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t >> LOGL, lx = t & (S::L - 1);
        v[k] = (!sparse || lcol[lx >> lt.log_tile_x])
                   ? mid[((((size_t)(lx >> log_panel)) * my + row0 + c) << log_panel) + (lx & cmask)]
                   : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t >> LOGL, lx = t & (S::L - 1);
        lds[c * S::STRIDE + lds_pos<S::PS>(lx)] = v[k];
        if constexpr (SPLIT) big = fmaxf(big, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    }
    // split products: scale the workgroup's data by a power of two into FP16 range
    // (applied as the first stage reads it); the block maximum's barrier also
    // completes the LDS writes above, as transform_all's first barrier does otherwise
    float unscale = 1.f, inv = 1.f;
    if constexpr (SPLIT) {
        const int e = range_exponent(block_max(big, scratch));
        inv = ldexpf(1.f, -e);
        unscale = ldexpf(1.f, e);
    }
    transform_all<LOGL, BATCH, NT, SPLIT>(lds, tw, w16, inv);
    // mx = L / 2 (the fine grid is twice the destination), so the epilogue's trip
    // count is a constant too: its table (and accumulated) loads go out together
    (void)mx;
    constexpr int MX = S::L / 2, HALF = MX / 2;
    constexpr int OUT = MX * BATCH / NT;
    float2 dxv[OUT], prev[OUT];
#pragma unroll
    for (int k = 0; k < OUT; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t / MX, ix = t - c * MX;
        dxv[k] = dx[ix];
        prev[k] = accumulate ? u2[(size_t)(row0 + c) * MX + ix] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < OUT; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t / MX, ix = t - c * MX;
        const int l = (ix - HALF) & (S::L - 1);
        float2 val = lds[c * S::STRIDE + lds_pos<S::PS>(l)];
        val = make_float2(val.x * unscale, val.y * unscale);
        const float2 r = cmul(cmul(val, dxv[k]), dy[row0 + c]);
        u2[(size_t)(row0 + c) * MX + ix] = make_float2(prev[k].x + r.x, prev[k].y + r.y);
    }
}

// ---- adjoint (type-2 direction) -------------------------------------------------
// The adjoint of the forward's two pruned passes: the kept modes, zero-padded
// to the fine grid, go through the unnormalised inverse-direction (exp(+i)) DFT,
// rows first, then columns.  exp(+i) transforms reuse the exp(-i) stages as
// conj(DFT(conj(x))): values are conjugated on the way into LDS and out of it.
// Mode m of a length-L transform sits at index m mod L; destination pixel ix
// is mode ix - mx/2.

// Adjoint pass 2: a workgroup takes BATCH rows of g2, multiplies by
// conj(Dx[ix] Dy[iy]) (the adjoint of the fused deconvolution and phase),
// zero-pads to nfx and writes the transformed rows to mid (my x nfx, row-major).
template <int LOGL, int BATCH, int NT, bool SPLIT>
__global__ void __launch_bounds__(NT) fft_adj_rows_kernel(const float2 *__restrict__ g2,
                                                          float2 *__restrict__ mid,
                                                          const float2 *__restrict__ tw,
                                                          const float2 *__restrict__ w16,
                                                          const float2 *__restrict__ dx,
                                                          const float2 *__restrict__ dy, int mx,
                                                          LiveTiles lt) {
    using S = Len<LOGL>;
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lcol[kMaxTileCols];
    const int row0 = blockIdx.x * BATCH;
    const bool sparse = live_cols(lt, lcol);
    const int half = mx >> 1;
    float big = 0.f;
    // every load in flight before the first LDS write
    constexpr int PER = S::L * BATCH / NT;
    float2 gv[PER], dv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t >> LOGL, l = t & (S::L - 1);
        const int m = l < S::L / 2 ? l : l - S::L;
        const int ix = m + half;
        const bool in = ix >= 0 && ix < mx;
        gv[k] = in ? g2[(size_t)(row0 + c) * mx + ix] : make_float2(0.f, 0.f);
        dv[k] = in ? dx[ix] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t >> LOGL, l = t & (S::L - 1);
        // conj(g conj(Dx Dy)) = conj(g) Dx Dy (zero outside the kept modes)
        const float2 v = cmul(cmul(make_float2(gv[k].x, -gv[k].y), dv[k]), dy[row0 + c]);
        lds[c * S::STRIDE + lds_pos<S::PS>(l)] = v;
        if constexpr (SPLIT) big = fmaxf(big, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    // split products: scale the workgroup's data by a power of two into FP16 range
    // (applied as the first stage reads it); the block maximum's barrier also
    // completes the LDS writes above, as transform_all's first barrier does otherwise
    float unscale = 1.f, inv = 1.f;
    if constexpr (SPLIT) {
        const int e = range_exponent(block_max(big, scratch));
        inv = ldexpf(1.f, -e);
        unscale = ldexpf(1.f, e);
    }
    transform_all<LOGL, BATCH, NT, SPLIT>(lds, tw, w16, inv);
    float2 *dst = mid + (size_t)row0 * S::L;
    for (int t = threadIdx.x; t < S::L * BATCH; t += NT) {
        const int c = t >> LOGL, l = t & (S::L - 1);
        if (sparse && !lcol[l >> lt.log_tile_x]) continue;   // a column the column pass skips
        const float2 v = lds[c * S::STRIDE + lds_pos<S::PS>(l)];
        dst[t] = make_float2(v.x * unscale, -v.y * unscale);
    }
}

// Adjoint pass 1: a workgroup takes BATCH adjacent columns of mid (the my kept
// rows), zero-pads to nfy and writes the transformed columns to the fine grid
// in its panel layout (one contiguous block per workgroup; with the binning's
// flags, only the cells of tiles some record reaches, which are all that the
// interpolation uses).  The 16 / BATCH
// panels that share 128-byte lines of mid rows run on one XCD.
template <int LOGL, int BATCH, int NT, bool SPLIT, int FP>
__global__ void __launch_bounds__(NT) fft_adj_cols_kernel(const float2 *__restrict__ mid,
                                                          float2 *__restrict__ fine,
                                                          const float2 *__restrict__ tw,
                                                          const float2 *__restrict__ w16,
                                                          int nfx, int my, int xcd_group,
                                                          LiveTiles lt) {
    using S = Len<LOGL>;
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lrow[kMaxTileRows];
    int pc = blockIdx.x;
    if (xcd_group > 1) {
        const int xcd = pc & 7, slot = pc >> 3;
        pc = ((slot / xcd_group) * 8 + xcd) * xcd_group + slot % xcd_group;
    }
    // with flags: a panel no record reaches is not needed at all, and in the others
    // only the cells of tiles some record reaches are stored
    if (!column_needed(lt, pc * BATCH)) return;
    const bool sparse = live_rows(lt, pc * BATCH, lrow);
    const int half = my >> 1;
    float big = 0.f;
    // every load in flight before the first LDS write
    constexpr int PER = S::L * BATCH / NT;
    float2 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int l = t / BATCH, c = t % BATCH;
        const int m = l < S::L / 2 ? l : l - S::L;
        const int ky = m + half;
        v[k] = (ky >= 0 && ky < my) ? mid[(size_t)ky * nfx + pc * BATCH + c] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * NT;
        const int l = t / BATCH, c = t % BATCH;
        const float2 w = make_float2(v[k].x, -v[k].y);
        lds[c * S::STRIDE + lds_pos<S::PS>(l)] = w;
        if constexpr (SPLIT) big = fmaxf(big, fmaxf(fabsf(w.x), fabsf(w.y)));
    }
    // split products: scale the workgroup's data by a power of two into FP16 range
    // (applied as the first stage reads it); the block maximum's barrier also
    // completes the LDS writes above, as transform_all's first barrier does otherwise
    float unscale = 1.f, inv = 1.f;
    if constexpr (SPLIT) {
        const int e = range_exponent(block_max(big, scratch));
        inv = ldexpf(1.f, -e);
        unscale = ldexpf(1.f, e);
    }
    transform_all<LOGL, BATCH, NT, SPLIT>(lds, tw, w16, inv);
    if constexpr (FP == BATCH) {
        float2 *dst = fine + (size_t)pc * S::L * BATCH;
        for (int t = threadIdx.x; t < S::L * BATCH; t += NT) {
            const int l = t / BATCH, c = t % BATCH;
            if (sparse && !lrow[l >> lt.log_tile_y]) continue;
            const float2 v = lds[c * S::STRIDE + lds_pos<S::PS>(l)];
            dst[t] = make_float2(v.x * unscale, -v.y * unscale);
        }
    } else {
        // the fine grid in panels of FP < BATCH columns (FP = 1: column-major)
        static_assert(FP == 1, "narrower fine-grid panels are single columns");
        float2 *dst = fine + (size_t)pc * S::L * BATCH;   // this workgroup's BATCH whole columns
        for (int t = threadIdx.x; t < S::L * BATCH; t += NT) {
            const int c = t >> LOGL, l = t & (S::L - 1);
            if (sparse && !lrow[l >> lt.log_tile_y]) continue;
            const float2 v = lds[c * S::STRIDE + lds_pos<S::PS>(l)];
            dst[t] = make_float2(v.x * unscale, -v.y * unscale);
        }
    }
}

// ---- passes whose first and last stages touch global memory directly ----------
// For lengths L = 16^a (256 and 4096 points: the first stage is a radix-16 stage)
// the first stage's four inputs per lane are loaded from global memory straight
// into the matrix-core lane layout, and the last stage's outputs (only the kept
// modes) are stored straight to global memory: the data crosses LDS a - 1 times
// instead of a + 1, with four barriers fewer per pass.

// This lane's inputs of the first radix-16 stage: element j + (g + 4 i) L/16 of
// transform c, read through load(c, e).
template <int LOGL, int BATCH, int NT, class Load>
__device__ __forceinline__ void first_inputs(Load load, float2 (&v)[StageBlocks<LOGL, BATCH, NT>::BPW][4]) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jj = lane & 15, wave = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int q = (wave * BPW + b) * 16 + jj;
        const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[b][i] = load(c, j + (g + 4 * i) * S::LQ);
    }
}

// Inputs of a stage with span NS from LDS, times this stage's twiddles, through
// the 16-point DFTs.
template <int LOGL, int BATCH, int NT, int NS, class Engine>
__device__ __forceinline__ void stage_read_run(const float2 *lds,
                                               const float4 (&t)[StageBlocks<LOGL, BATCH, NT>::BPW][2],
                                               float2 (&v)[StageBlocks<LOGL, BATCH, NT>::BPW][4],
                                               const Engine &eng) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jj = lane & 15, wave = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int q = (wave * BPW + b) * 16 + jj;
        const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
        const float2 *col = lds + c * S::STRIDE;
        if constexpr (S::LQ >= 64) {
            const float2 *src = col + lds_pos<S::PS>(j + g * S::LQ);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = src[i * (4 * S::LQ + 64)];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = col[lds_pos<S::PS>(j + (g + 4 * i) * S::LQ)];
        }
        if constexpr (NS > 1) {
            v[b][0] = cmul(v[b][0], make_float2(t[b][0].x, t[b][0].y));
            v[b][1] = cmul(v[b][1], make_float2(t[b][0].z, t[b][0].w));
            v[b][2] = cmul(v[b][2], make_float2(t[b][1].x, t[b][1].y));
            v[b][3] = cmul(v[b][3], make_float2(t[b][1].z, t[b][1].w));
        }
        eng.run(v[b]);
    }
}

// A stage's outputs (span NS) to their Stockham positions in LDS.
template <int LOGL, int BATCH, int NT, int NS>
__device__ __forceinline__ void stage_write(float2 *lds, const float2 (&v)[StageBlocks<LOGL, BATCH, NT>::BPW][4]) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jj = lane & 15, wave = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int q = (wave * BPW + b) * 16 + jj;
        const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
        const int k = j & (NS - 1);
        const int base = (j - k) * 16 + k;
        float2 *col = lds + c * S::STRIDE;
        if constexpr (NS >= 64 && (4 * NS) % S::LQ == 0) {
            float2 *dst = col + lds_pos<S::PS>(base + g * NS);
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[i * (4 * NS + ((4 * NS) >> S::PS) * 16)] = v[b][i];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) col[lds_pos<S::PS>(base + (g + 4 * i) * NS)] = v[b][i];
        }
    }
}

// Stages STAGE .. a-1 (span 16^STAGE, twiddles tcur already in registers); the
// last one hands its outputs to store(c, l, value): output l of transform c.
template <int LOGL, int BATCH, int NT, int STAGE, class Engine, class Store>
__device__ __forceinline__ void direct_rest(float2 *lds, const float4 *tw4, const Engine &eng,
                                            const float4 (&tcur)[StageBlocks<LOGL, BATCH, NT>::BPW][2],
                                            Store store, float unscale) {
    using S = Len<LOGL>;
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    constexpr int NS = 1 << (4 * STAGE);
    float2 v[BPW][4];
    stage_read_run<LOGL, BATCH, NT, NS, Engine>(lds, tcur, v, eng);
    if constexpr (STAGE + 1 < S::N16) {
        float4 tnext[BPW][2];
        load_twiddles<LOGL, BATCH, NT, NS * 16>(stage_table<LOGL>(tw4, STAGE + 1), tnext);
        __syncthreads();
        stage_write<LOGL, BATCH, NT, NS>(lds, v);
        __syncthreads();
        direct_rest<LOGL, BATCH, NT, STAGE + 1, Engine, Store>(lds, tw4, eng, tnext, store, unscale);
    } else {
        // span NS = L/16: output p = g + 4 i of instance j is element j + p NS
        const int lane = threadIdx.x & 63;
        const int g = lane >> 4, jj = lane & 15, wave = threadIdx.x >> 6;
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int q = (wave * BPW + b) * 16 + jj;
            const int c = q >> S::LOGLQ, j = q & (S::LQ - 1);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                store(c, j + (g + 4 * i) * NS, make_float2(v[b][i].x * unscale, v[b][i].y * unscale));
        }
    }
}

// The workgroup's BATCH transforms of length L = 16^a: inputs through load(c, e),
// the kept outputs through store(c, l, value).  With SPLIT the inputs are scaled by
// the power of two that brings the workgroup's largest |Re|, |Im| to at most 1
// (and the outputs scaled back).
template <int LOGL, int BATCH, int NT, bool SPLIT, class Load, class Store>
__device__ __forceinline__ void transform_direct(float2 *lds, const float2 *tw, const float2 *w16,
                                                 float *scratch, Load load, Store store) {
    using S = Len<LOGL>;
    static_assert(S::R0 == 1 && S::N16 >= 2, "lengths 16^a, a >= 2");
    constexpr int BPW = StageBlocks<LOGL, BATCH, NT>::BPW;
    const float4 *tw4 = reinterpret_cast<const float4 *>(tw);
    const int lane = threadIdx.x & 63;
    float2 v[BPW][4];
    first_inputs<LOGL, BATCH, NT>(load, v);
    float4 t1[BPW][2];
    load_twiddles<LOGL, BATCH, NT, 16>(stage_table<LOGL>(tw4, 1), t1);
    float unscale = 1.f;
    if constexpr (SPLIT) {
        float big = 0.f;
#pragma unroll
        for (int b = 0; b < BPW; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) big = fmaxf(big, fmaxf(fabsf(v[b][i].x), fabsf(v[b][i].y)));
        const int e = range_exponent(block_max(big, scratch));
        const float inv = ldexpf(1.f, -e);
        unscale = ldexpf(1.f, e);
#pragma unroll
        for (int b = 0; b < BPW; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[b][i] = make_float2(v[b][i].x * inv, v[b][i].y * inv);
    }
    using Engine = typename std::conditional<SPLIT, Dft16Split16, Dft16Valu>::type;
    Engine eng;
    eng.init(w16, lane >> 4, lane & 15);
#pragma unroll
    for (int b = 0; b < BPW; ++b) eng.run(v[b]);
    stage_write<LOGL, BATCH, NT, 1>(lds, v);
    __syncthreads();
    direct_rest<LOGL, BATCH, NT, 1, Engine, Store>(lds, tw4, eng, t1, store, unscale);
}

// Pass 1 for L = 16^a: a workgroup transforms one panel of BATCH adjacent columns.
// mid's panels hold MP >= BATCH columns: the MP / BATCH workgroups that fill one
// panel (each writing its columns' pieces of the panel's lines) run on one XCD when
// xcd_pair is set, so that its L2 merges the pieces before they reach HBM.
template <int LOGL, int BATCH, int NT, bool SPLIT, int MP>
__global__ void __launch_bounds__(NT) fft_pass1_direct_kernel(const float2 *__restrict__ fine,
                                                              float2 *__restrict__ mid,
                                                              const float2 *__restrict__ tw,
                                                              const float2 *__restrict__ w16, int my,
                                                              LiveTiles lt, int xcd_pair) {
    using S = Len<LOGL>;
    static_assert(MP % BATCH == 0, "mid panels hold whole column batches");
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lrow[kMaxTileRows];
    int pc = blockIdx.x;
    if (MP > BATCH && xcd_pair) {
        constexpr int G = MP / BATCH;
        const int xcd = pc & 7, slot = pc >> 3;
        pc = ((slot / G) * 8 + xcd) * G + slot % G;
    }
    const float2 *src = fine + (size_t)pc * S::L * BATCH;
    const int x0 = pc * BATCH;
    float2 *dst = mid + (size_t)(x0 / MP) * my * MP + x0 % MP;   // this batch's columns of its mid panel
    const int half = my >> 1;
    if (!column_needed(lt, pc * BATCH)) return;
    const bool sparse = live_rows(lt, pc * BATCH, lrow);
    transform_direct<LOGL, BATCH, NT, SPLIT>(
        lds, tw, w16, scratch,
        [&](int c, int e) {
            return (!sparse || lrow[e >> lt.log_tile_y]) ? src[e * BATCH + c] : make_float2(0.f, 0.f);
        },
        [&](int c, int l, float2 val) {
            const int ky = (l + half) & (S::L - 1);
            if (ky < my) dst[ky * MP + c] = val;
        });
}

// Pass 2 for L = 16^a: a workgroup transforms BATCH rows of mid; fused deconvolution
// and destination phase (mx = L / 2).
template <int LOGL, int BATCH, int NT, bool SPLIT>
__global__ void __launch_bounds__(NT) fft_pass2_direct_kernel(const float2 *__restrict__ mid,
                                                              float2 *__restrict__ u2,
                                                              const float2 *__restrict__ tw,
                                                              const float2 *__restrict__ w16,
                                                              const float2 *__restrict__ dx,
                                                              const float2 *__restrict__ dy, int my,
                                                              int log_panel, int xcd_group, int accumulate,
                                                              LiveTiles lt) {
    using S = Len<LOGL>;
    extern __shared__ float2 lds[];
    __shared__ float scratch[NT / 64];
    __shared__ uint8_t lcol[kMaxTileCols];
    int g = blockIdx.x;
    if (xcd_group > 1) {
        const int xcd = g & 7, slot = g >> 3;
        g = ((slot / xcd_group) * 8 + xcd) * xcd_group + slot % xcd_group;
    }
    const int row0 = g * BATCH;
    const int cmask = (1 << log_panel) - 1;
    constexpr int MX = S::L / 2, HALF = MX / 2;
    const bool sparse = live_cols(lt, lcol);
    transform_direct<LOGL, BATCH, NT, SPLIT>(
        lds, tw, w16, scratch,
        [&](int c, int e) {
            return (!sparse || lcol[e >> lt.log_tile_x])
                       ? mid[((((size_t)(e >> log_panel)) * my + row0 + c) << log_panel) + (e & cmask)]
                       : make_float2(0.f, 0.f);
        },
        [&](int c, int l, float2 val) {
            const int ix = (l + HALF) & (S::L - 1);
            if (ix < MX) {
                float2 *o = u2 + (size_t)(row0 + c) * MX + ix;
                const float2 r = cmul(cmul(val, dx[ix]), dy[row0 + c]);
                *o = accumulate ? make_float2(o->x + r.x, o->y + r.y) : r;
            }
        });
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

// Threads per workgroup for BATCH transforms of length 2^LOGL: one wave per
// 16-instance block up to 8 waves, then several blocks per wave.
template <int LOGL, int BATCH>
constexpr int threads_for() {
    constexpr int blocks = BATCH * (1 << LOGL) / 256;
    constexpr int nt = blocks <= 8 ? 64 * blocks : 512;
    // the kernels' loaders give every thread exactly L * BATCH / NT elements
    static_assert((BATCH << LOGL) % nt == 0, "whole elements per thread");
    return nt;
}

template <int LOGL, int BATCH, bool SPLIT, int MP = BATCH>
hipError_t launch1(const FftShape &sh, const float2 *fine, float2 *mid, const float2 *tw,
                   const float2 *w16, int nfx, int my, const LiveTiles &lt, hipStream_t s) {
    (void)sh;
    constexpr int NT = threads_for<LOGL, BATCH>();
    const size_t lds = (size_t)BATCH * Len<LOGL>::STRIDE * sizeof(float2);
    static thread_local size_t enabled = 0;
    if constexpr (LOGL % 4 == 0 && LOGL >= 8) {
        auto k = fft_pass1_direct_kernel<LOGL, BATCH, NT, SPLIT, MP>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        const int groups = nfx / BATCH;
        const int xcd_pair = (MP > BATCH && groups % (8 * (MP / BATCH)) == 0) ? 1 : 0;
        hipLaunchKernelGGL(k, dim3(groups), dim3(NT), lds, s, fine, mid, tw, w16, my, lt, xcd_pair);
    } else {
        auto k = fft_pass1_kernel<LOGL, BATCH, NT, SPLIT, MP>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        const int groups = nfx / BATCH;
        const int xcd_pair = (MP > BATCH && groups % (8 * (MP / BATCH)) == 0) ? 1 : 0;
        hipLaunchKernelGGL(k, dim3(groups), dim3(NT), lds, s, fine, mid, tw, w16, my, lt, xcd_pair);
    }
    return hipGetLastError();
}

template <int LOGL, int BATCH, bool SPLIT>
hipError_t launch2(const FftShape &sh, const float2 *mid, float2 *u2, const float2 *tw,
                   const float2 *w16, const float2 *dx, const float2 *dy, int mx, int my,
                   int log_panel, int accumulate, const LiveTiles &lt, hipStream_t s) {
    constexpr int NT = threads_for<LOGL, BATCH>();
    const size_t lds = (size_t)BATCH * Len<LOGL>::STRIDE * sizeof(float2);
    static thread_local size_t enabled = 0;
    (void)sh;
    const int groups = my / BATCH;
    const int rows_per_line = 16 >> log_panel;   // rows of mid that share a 128-byte line
    const int g = rows_per_line > BATCH ? rows_per_line / BATCH : 1;
    const int xcd_group = (g > 1 && groups % (8 * g) == 0) ? g : 1;
    if constexpr (LOGL % 4 == 0 && LOGL >= 8) {
        auto k = fft_pass2_direct_kernel<LOGL, BATCH, NT, SPLIT>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        if (mx != Len<LOGL>::L / 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k, dim3(groups), dim3(NT), lds, s, mid, u2, tw, w16, dx, dy, my, log_panel,
                           xcd_group, accumulate, lt);
    } else {
        auto k = fft_pass2_kernel<LOGL, BATCH, NT, SPLIT>;
        hipError_t e = allow_lds((const void *)k, lds, enabled);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(groups), dim3(NT), lds, s, mid, u2, tw, w16, dx, dy, mx, my, log_panel,
                           xcd_group, accumulate, lt);
    }
    return hipGetLastError();
}

template <int LOGL, int BATCH, bool SPLIT>
hipError_t launch_adj2(const float2 *g2, float2 *mid, const float2 *tw, const float2 *w16,
                       const float2 *dx, const float2 *dy, int mx, int my, const LiveTiles &lt,
                       hipStream_t s) {
    constexpr int NT = threads_for<LOGL, BATCH>();
    const size_t lds = (size_t)BATCH * Len<LOGL>::STRIDE * sizeof(float2);
    static thread_local size_t enabled = 0;
    auto k = fft_adj_rows_kernel<LOGL, BATCH, NT, SPLIT>;
    hipError_t e = allow_lds((const void *)k, lds, enabled);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(my / BATCH), dim3(NT), lds, s, g2, mid, tw, w16, dx, dy, mx, lt);
    return hipGetLastError();
}

template <int LOGL, int BATCH, bool SPLIT, int FP = BATCH>
hipError_t launch_adj1(const float2 *mid, float2 *fine, const float2 *tw, const float2 *w16,
                       int nfx, int my, const LiveTiles &lt, hipStream_t s) {
    constexpr int NT = threads_for<LOGL, BATCH>();
    const size_t lds = (size_t)BATCH * Len<LOGL>::STRIDE * sizeof(float2);
    static thread_local size_t enabled = 0;
    auto k = fft_adj_cols_kernel<LOGL, BATCH, NT, SPLIT, FP>;
    hipError_t e = allow_lds((const void *)k, lds, enabled);
    if (e != hipSuccess) return e;
    const int groups = nfx / BATCH;
    const int g = BATCH < 16 ? 16 / BATCH : 1;   // panels per 128-byte line of a mid row
    const int xcd_group = (g > 1 && groups % (8 * g) == 0) ? g : 1;
    hipLaunchKernelGGL(k, dim3(groups), dim3(NT), lds, s, mid, fine, tw, w16, nfx, my, xcd_group, lt);
    return hipGetLastError();
}

template <bool SPLIT>
hipError_t dispatch_adj2(int len, const float2 *g2, float2 *mid, const float2 *tw, const float2 *w16,
                         const float2 *dx, const float2 *dy, int mx, int my, const LiveTiles &lt, hipStream_t s) {
    switch (__builtin_ctz(len)) {
        case 5: return launch_adj2<5, 8, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 6: return launch_adj2<6, 4, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 7: return launch_adj2<7, 2, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 8: return launch_adj2<8, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 9: return launch_adj2<9, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 10: return launch_adj2<10, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 11: return launch_adj2<11, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 12: return launch_adj2<12, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 13: return launch_adj2<13, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        case 14: return launch_adj2<14, 1, SPLIT>(g2, mid, tw, w16, dx, dy, mx, my, lt, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool SPLIT>
hipError_t dispatch_adj1(int len, const float2 *mid, float2 *fine, const float2 *tw,
                         const float2 *w16, int nfx, int my, const LiveTiles &lt, hipStream_t s) {
    switch (__builtin_ctz(len)) {
        case 5: return launch_adj1<5, 16, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 6: return launch_adj1<6, 16, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 7: return launch_adj1<7, 16, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 8: return launch_adj1<8, 16, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 9: return launch_adj1<9, 16, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 10: return launch_adj1<10, 8, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 11: return launch_adj1<11, 4, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 12: return launch_adj1<12, 2, SPLIT, 1>(mid, fine, tw, w16, nfx, my, lt, s);
        case 13: return launch_adj1<13, 1, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        case 14: return launch_adj1<14, 1, SPLIT>(mid, fine, tw, w16, nfx, my, lt, s);
        default: return hipErrorInvalidValue;
    }
}

// Batch sizes used per length (the same as fft_batch_pass1/2): pass 1 holds up to
// 70 KB of LDS -- 16 columns up to 512 points, then 8, 4, and one column from 4096
// up.  At 4096 and 8192 mid keeps panels of two and four columns (fft_mid_panel),
// each filled by that many one-column workgroups on one XCD: the row pass gathers
// 16- and 32-byte pieces of mid's lines instead of 8 (15 us less at the 4096^2 fine
// grid, 35 us at 8192^2, where pass 1 pays 15 us of it back) while pass 1 keeps one
// column per workgroup.  The adjoint's column pass takes two columns at 4096 and
// stores them column-major.  Pass 2 uses one row unless the row is shorter than 256.
template <bool SPLIT>
hipError_t dispatch1(const FftShape &sh, const float2 *fine, float2 *mid, const float2 *tw,
                     const float2 *w16, int nfx, int my, const LiveTiles &lt, hipStream_t s) {
    const int log = __builtin_ctz(sh.L);
    switch (log) {
        case 5: return launch1<5, 16, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 6: return launch1<6, 16, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 7: return launch1<7, 16, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 8: return launch1<8, 16, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 9: return launch1<9, 16, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 10: return launch1<10, 8, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 11: return launch1<11, 4, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 12: return launch1<12, 1, SPLIT, 2>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 13: return launch1<13, 1, SPLIT, 4>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        case 14: return launch1<14, 1, SPLIT>(sh, fine, mid, tw, w16, nfx, my, lt, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool SPLIT>
hipError_t dispatch2(const FftShape &sh, int log_panel, const float2 *mid, float2 *u2, const float2 *tw,
                     const float2 *w16, const float2 *dx, const float2 *dy, int mx, int my,
                     int accumulate, const LiveTiles &lt, hipStream_t s) {
    const int log = __builtin_ctz(sh.L);
    switch (log) {
        case 5: return launch2<5, 8, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 6: return launch2<6, 4, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 7: return launch2<7, 2, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 8: return launch2<8, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 9: return launch2<9, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 10: return launch2<10, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 11: return launch2<11, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 12: return launch2<12, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 13: return launch2<13, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        case 14: return launch2<14, 1, SPLIT>(sh, mid, u2, tw, w16, dx, dy, mx, my, log_panel, accumulate, lt, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int fft_batch_pass1(int len) {
    const int log = __builtin_ctz(len);
    return log <= 9 ? 16 : log == 10 ? 8 : log == 11 ? 4 : 1;
}

int fft_mid_panel(int len) {
    const int log = __builtin_ctz(len);
    return log == 12 ? 2 : log == 13 ? 4 : fft_batch_pass1(len);
}

int fft_batch_pass2(int len) {
    const int log = __builtin_ctz(len);
    return log == 5 ? 8 : log == 6 ? 4 : log == 7 ? 2 : 1;
}

size_t fft_lds_bytes(int len, int batch) {
    const int log = __builtin_ctz(len);
    const int lq = len / 16;
    const int ps = lq > 16 ? log - 4 : 4;
    return (size_t)batch * (len + (len >> ps) * 16) * sizeof(float2);
}

int fft_max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

hipError_t launch_fft_pass1(const FftShape &sh, int split16, const float2 *fine, float2 *mid,
                            const float2 *tw, const float2 *w16, int nfx, int my, const LiveTiles &lt,
                            hipStream_t s) {
    if (lt.flag && (lt.nty > kMaxTileRows || lt.nty <= 0)) return hipErrorInvalidValue;
    if (split16) return dispatch1<true>(sh, fine, mid, tw, w16, nfx, my, lt, s);
    return dispatch1<false>(sh, fine, mid, tw, w16, nfx, my, lt, s);
}

hipError_t launch_fft_pass2(const FftShape &sh, int log_panel, int split16, const float2 *mid,
                            float2 *u2, const float2 *tw, const float2 *w16, const float2 *dx,
                            const float2 *dy, int mx, int my, int accumulate, const LiveTiles &lt,
                            hipStream_t s) {
    if (lt.flag && (lt.ntx > kMaxTileCols || lt.ntx <= 0)) return hipErrorInvalidValue;
    if (split16) return dispatch2<true>(sh, log_panel, mid, u2, tw, w16, dx, dy, mx, my, accumulate, lt, s);
    return dispatch2<false>(sh, log_panel, mid, u2, tw, w16, dx, dy, mx, my, accumulate, lt, s);
}

hipError_t launch_fft_adj_rows(int len, int split16, const float2 *g2, float2 *mid, const float2 *tw,
                               const float2 *w16, const float2 *dx, const float2 *dy, int mx, int my,
                               const LiveTiles &lt, hipStream_t s) {
    if (lt.flag && (lt.ntx > kMaxTileCols || lt.ntx <= 0)) return hipErrorInvalidValue;
    if (split16) return dispatch_adj2<true>(len, g2, mid, tw, w16, dx, dy, mx, my, lt, s);
    return dispatch_adj2<false>(len, g2, mid, tw, w16, dx, dy, mx, my, lt, s);
}

hipError_t launch_fft_adj_cols(int len, int split16, const float2 *mid, float2 *fine,
                               const float2 *tw, const float2 *w16, int nfx, int my, const LiveTiles &lt,
                               hipStream_t s) {
    if (lt.flag && (lt.nty > kMaxTileRows || lt.nty <= 0)) return hipErrorInvalidValue;
    if (split16) return dispatch_adj1<true>(len, mid, fine, tw, w16, nfx, my, lt, s);
    return dispatch_adj1<false>(len, mid, fine, tw, w16, nfx, my, lt, s);
}

}  // namespace asf
