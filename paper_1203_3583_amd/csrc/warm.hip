// Kernels of the learned warm start (include/asf_warm.h): a small convolutional
// encoder-decoder that maps (target intensity, surface height) to a source
// phase, trained through the forward and adjoint of the diffraction method.
//
// The convolutions are implicit GEMMs on the matrix cores,
// v_mfma_f32_16x16x16_bf16 and, for 32-channel slices, v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation):
//   forward  D[pixel][cout] = sum_k A[pixel][k] W[k][cout],  k = (ky 3 + kx) cin + ci,
//            A[p][k] the input pixel p shifted by (ky-1, kx-1) (zero outside);
//   wgrad    D[cout][k]     = sum_p dOut[p][cout] A[p][k]   (contraction over pixels);
//   input gradient: the forward with flipped, transposed weights.
// Channels-last storage makes every operand fetch contiguous: in a 16 x 16 x 16
// step, lane l (row or column l % 16, k group l / 16) reads four consecutive
// channels of one pixel (16 bytes of FP32 activations) or four consecutive k of
// one weight row (8 bytes of BF16).  The accumulator tile of lane l holds rows
// 4 (l / 16) + i, column l % 16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asf_warm.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ v4s bf16x4(float4 v) {
    v4s r;
    r[0] = bf16(v.x);
    r[1] = bf16(v.y);
    r[2] = bf16(v.z);
    r[3] = bf16(v.w);
    return r;
}

// ---- forward convolution, direct (small layers) -----------------------------------
// A wave computes 16 PB consecutive pixels (flattened b, y, x) x 32 output
// channels: PB x 2 accumulator tiles, reading its operands straight from
// memory (PB = 1 for the small layers this kernel serves: more waves).  Four
// waves per workgroup, on consecutive pixel tiles of the same channel block; no
// LDS, no barriers.  The contraction runs over (tap, 16
// channels) steps, two per iteration with all their loads issued first.
constexpr int kConvWaves = 4;

template <int PB>
__global__ __launch_bounds__(64 * kConvWaves) void conv3x3_kernel(
    const float *__restrict__ in, const uint16_t *__restrict__ w, const float *__restrict__ bias,
    float *__restrict__ out, int B, int H, int W, int cin, int cout, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npix = (int64_t)B * H * W;
    const int64_t p0 = ((int64_t)blockIdx.x * kConvWaves + wave) * (16 * PB);
    if (p0 >= npix) return;   // uniform over the wave
    const int co0 = blockIdx.y * 32;
    const int r = lane & 15, g = lane >> 4;
    // the pixels whose A rows this lane supplies
    int py[PB], px[PB];
    int64_t pimg[PB];   // b H W of the pixel's image, or -1 past the end
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
        const int64_t p = p0 + pb * 16 + r;
        if (p < npix) {
            const int64_t bi = p / ((int64_t)H * W);
            const int rest = (int)(p - bi * H * W);
            py[pb] = rest / W;
            px[pb] = rest - py[pb] * W;
            pimg[pb] = bi * H * W;
        } else {
            py[pb] = px[pb] = 0;
            pimg[pb] = -1;
        }
    }
    v4f acc[PB][2];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[pb][cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    const int kin = 9 * cin;
    const uint16_t *wrow0 = w + (size_t)(co0 + r) * kin;
    const uint16_t *wrow1 = w + (size_t)(co0 + 16 + r) * kin;
    const int steps = 9 * (cin >> 4);
    int tap = 0, c0 = 0;   // (tap, first channel) of step s
    for (int s = 0; s < steps; s += 2) {
        float4 v[2][PB];
        v4s b0[2], b1[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool live = s + h < steps;   // uniform over the wave
            const int ty = tap / 3;
            const int dy = ty - 1, dx = tap - 3 * ty - 1;
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) {
                const int yy = py[pb] + dy, xx = px[pb] + dx;
                const bool ok = live && pimg[pb] >= 0 && yy >= 0 && yy < H && xx >= 0 && xx < W;
                v[h][pb] = ok ? *reinterpret_cast<const float4 *>(in + (size_t)(pimg[pb] + (int64_t)yy * W + xx) * cin +
                                                                  c0 + g * 4)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            const int k = tap * cin + c0 + g * 4;
            b0[h] = live ? *reinterpret_cast<const v4s *>(wrow0 + k) : (v4s){0, 0, 0, 0};
            b1[h] = live ? *reinterpret_cast<const v4s *>(wrow1 + k) : (v4s){0, 0, 0, 0};
            c0 += 16;
            if (c0 == cin) {
                c0 = 0;
                ++tap;
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (s + h >= steps) break;   // uniform
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) {
                const v4s a = bf16x4(v[h][pb]);
                acc[pb][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b0[h], acc[pb][0], 0, 0, 0);
                acc[pb][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b1[h], acc[pb][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int co = co0 + cb * 16 + r;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = p0 + pb * 16 + g * 4 + i;
                if (p >= npix) continue;
                float v = acc[pb][cb][i] + bv;
                if (relu) v = fmaxf(v, 0.f);
                out[p * cout + co] = v;
            }
    }
}

// ---- forward convolution, LDS-tiled ---------------------------------------------
// Large layers: a workgroup owns an 8 x 32 pixel tile of one image and 32 output
// channels.  Per 16-channel slice of the input it stages the tile plus its
// one-pixel halo (BF16, [row][column][16 channels]) and the slice's weights
// (BF16, [tap][cout][16 channels]) in LDS, then every wave (two rows of the tile,
// 4 x 2 accumulator tiles) runs the nine taps out of LDS: each input value is
// fetched from memory once per workgroup instead of once per tap.  A lane's
// 8-byte LDS reads (4 channels of one pixel, or of one weight row) cover 512
// contiguous bytes per wave: no bank conflicts.
constexpr int kTH = 8, kTW = 32;                 // output tile
constexpr int kHH = kTH + 2, kHWd = kTW + 2;     // tile with halo

__global__ __launch_bounds__(256) void conv3x3_tiled_kernel(
    const float *__restrict__ in, const uint16_t *__restrict__ w, const float *__restrict__ bias,
    float *__restrict__ out, int H, int W, int cin, int cout, int relu, int tiles_x, int tiles_y) {
    __shared__ __align__(16) uint16_t halo[kHH * kHWd * 16];
    __shared__ __align__(16) uint16_t wl[9 * 32 * 16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int t = blockIdx.x;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int b = t / tiles_y;
    const int y0 = ty * kTH, x0 = tx * kTW;
    const int co0 = blockIdx.y * 32;
    const int r = lane & 15, g = lane >> 4;
    const size_t img = (size_t)b * H * W;
    v4f acc[4][2];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) acc[pb][0] = acc[pb][1] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cin; c0 += 16) {
        __syncthreads();   // the previous slice has been read
        // the tile and halo: kHH x kHWd pixels x 4 groups of 4 channels
        for (int i = tid; i < kHH * kHWd * 4; i += 256) {
            const int q = i & 3, pix = i >> 2;
            const int hy = pix / kHWd, hx = pix - hy * kHWd;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                v = *reinterpret_cast<const float4 *>(in + (img + (size_t)yy * W + xx) * cin + c0 + 4 * q);
            *reinterpret_cast<v4s *>(halo + pix * 16 + 4 * q) = bf16x4(v);
        }
        // the slice's weights: 32 couts x 9 taps x 16 channels, 8 per load
        for (int i = tid; i < 32 * 9 * 2; i += 256) {
            const int hf = i & 1, rest = i >> 1;
            const int tap = rest % 9, co = rest / 9;
            const uint4 v = *reinterpret_cast<const uint4 *>(w + (size_t)(co0 + co) * 9 * cin + tap * cin + c0 + 8 * hf);
            *reinterpret_cast<uint4 *>(wl + (tap * 32 + co) * 16 + 8 * hf) = v;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;   // halo offsets of the tap
            const v4s bw0 = *reinterpret_cast<const v4s *>(wl + (tap * 32 + r) * 16 + 4 * g);
            const v4s bw1 = *reinterpret_cast<const v4s *>(wl + (tap * 32 + 16 + r) * 16 + 4 * g);
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int ly = 2 * wave + (pb >> 1), lx = (pb & 1) * 16 + r;
                const v4s a = *reinterpret_cast<const v4s *>(halo + ((ly + dy) * kHWd + lx + dx) * 16 + 4 * g);
                acc[pb][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw0, acc[pb][0], 0, 0, 0);
                acc[pb][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw1, acc[pb][1], 0, 0, 0);
            }
        }
    }
    // accumulator rows are pixels 4 g + i of the block, column r the output channel
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int co = co0 + cb * 16 + r;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + 2 * wave + (pb >> 1), x = x0 + (pb & 1) * 16 + 4 * g + i;
                if (y >= H || x >= W) continue;
                float v = acc[pb][cb][i] + bv;
                if (relu) v = fmaxf(v, 0.f);
                out[(img + (size_t)y * W + x) * cout + co] = v;
            }
    }
}

// ---- forward convolution, LDS-tiled, 32-channel slices -------------------------
// As conv3x3_tiled_kernel, for layers whose input channels come in multiples of
// 32: each slice stages 32 channels (BF16 tile and halo [row][column][32], weights
// [tap][cout][32]) and a tap's products are v_mfma_f32_16x16x32_bf16, gfx950's
// double-K BF16 instruction (half the matrix instructions and half the slices of
// the 16-channel kernel).  A lane's operands are 8 consecutive channels (16 bytes)
// of one pixel or of one weight row, the same channels in both operands.  The
// tile is TH x 32 pixels: TH = 8 where a layer has enough tiles to give every CU
// four workgroups, else 4 or 2 rows, so that the deep, small layers still spread
// over the whole chip (a 128^2 layer, 384 -> 128 channels: 0.089 ms with 8-row
// tiles, 0.060 ms with 2-row tiles; a 512^2 layer, 32 -> 32: 0.021 against 0.027).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int64_t kConvWorkgroupsWanted = 1024;   // four per CU

// The input of a 32-channel-slice convolution, channels-last: one tensor, or the
// decoder's concatenation read in place -- the 2x nearest-neighbour upsampling of a
// half-size tensor's c_low channels, then a full-size tensor's cin - c_low channels
// (c_low a multiple of 32, so every slice lies in one of the two).
struct ConvInput {
    const float *in;     // [B][H][W][cin], or NULL for the concatenation
    const float *low;    // [B][H/2][W/2][c_low]
    const float *skip;   // [B][H][W][cin - c_low]
    int c_low;
    // channels c0 .. c0 + 3 of pixel (b, y, x)
    __device__ __forceinline__ const float4 *at(size_t b, int y, int x, int H, int W, int cin, int c0) const {
        const float *p;
        if (in) p = in + ((b * H + y) * W + x) * cin + c0;
        else if (c0 < c_low) p = low + ((b * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1)) * c_low + c0;
        else p = skip + ((b * H + y) * W + x) * (cin - c_low) + (c0 - c_low);
        return reinterpret_cast<const float4 *>(p);
    }
};

template <int TH>
__global__ __launch_bounds__(256) void conv3x3_tiled32_kernel(
    ConvInput src, const uint16_t *__restrict__ w, const float *__restrict__ bias,
    float *__restrict__ out, int H, int W, int cin, int cout, int relu, int tiles_x, int tiles_y) {
    constexpr int HH = TH + 2;
    constexpr int BPW = TH / 2;            // 16-pixel blocks per wave (two per tile row)
    __shared__ __align__(16) uint16_t halo[HH * kHWd * 32];
    __shared__ __align__(16) uint16_t wl[9 * 32 * 32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int t = blockIdx.x;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int b = t / tiles_y;
    const int y0 = ty * TH, x0 = tx * kTW;
    const int co0 = blockIdx.y * 32;
    const int r = lane & 15, g = lane >> 4;
    const size_t img = (size_t)b * H * W;
    v4f acc[BPW][2];
#pragma unroll
    for (int pb = 0; pb < BPW; ++pb) acc[pb][0] = acc[pb][1] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cin; c0 += 32) {
        __syncthreads();   // the previous slice has been read
        for (int i = tid; i < HH * kHWd * 8; i += 256) {
            const int q = i & 7, pix = i >> 3;
            const int hy = pix / kHWd, hx = pix - hy * kHWd;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = *src.at(b, yy, xx, H, W, cin, c0 + 4 * q);
            *reinterpret_cast<v4s *>(halo + pix * 32 + 4 * q) = bf16x4(v);
        }
        for (int i = tid; i < 32 * 9 * 4; i += 256) {
            const int qq = i & 3, rest = i >> 2;
            const int tap = rest % 9, co = rest / 9;
            const uint4 v = *reinterpret_cast<const uint4 *>(w + (size_t)(co0 + co) * 9 * cin + tap * cin + c0 + 8 * qq);
            *reinterpret_cast<uint4 *>(wl + (tap * 32 + co) * 32 + 8 * qq) = v;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            const v8bf bw0 = *reinterpret_cast<const v8bf *>(wl + (tap * 32 + r) * 32 + 8 * g);
            const v8bf bw1 = *reinterpret_cast<const v8bf *>(wl + (tap * 32 + 16 + r) * 32 + 8 * g);
#pragma unroll
            for (int pb = 0; pb < BPW; ++pb) {
                const int k = wave * BPW + pb;
                const int ly = k >> 1, lx = (k & 1) * 16 + r;
                const v8bf a = *reinterpret_cast<const v8bf *>(halo + ((ly + dy) * kHWd + lx + dx) * 32 + 8 * g);
                acc[pb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw0, acc[pb][0], 0, 0, 0);
                acc[pb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw1, acc[pb][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int co = co0 + cb * 16 + r;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int pb = 0; pb < BPW; ++pb) {
            const int k = wave * BPW + pb;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + (k >> 1), x = x0 + (k & 1) * 16 + 4 * g + i;
                if (y >= H || x >= W) continue;
                float v = acc[pb][cb][i] + bv;
                if (relu) v = fmaxf(v, 0.f);
                out[(img + (size_t)y * W + x) * cout + co] = v;
            }
        }
    }
}

// ---- weight gradient ----------------------------------------------------------
// A wave computes a 32 (cout) x 16 (k) block of dw over a chunk of pixels and
// adds it to dw with FP32 atomics.  k = (tap, c0 .. c0+15): the block covers 16
// consecutive input channels of one tap; a wave takes kKB such blocks, which
// share its dout loads.  Short chunks give the deep, small layers enough waves;
// two 16-pixel steps per iteration keep their loads in flight together.
// pixels per wave: longer chunks mean fewer dw atomics, shorter ones more waves
// (a 512^2 layer, 96 -> 32 channels: 0.198 ms with 512, 0.261 with 256; 512^2,
// 16 -> 32: 0.047 ms with 256, 0.062 with 512)
constexpr int kWgradChunkSmall = 256;
constexpr int kWgradChunkLarge = 512;
constexpr int kMaxWgradPix = 1 << 22;   // B H W below this: pixel coordinates by float division

// Pixel p -> (b H W, y, x) for p < 2^22: a float estimate of each quotient, off by
// at most one (relative error below 2^-23 on a value below 2^22), then one
// correction step.
__device__ __forceinline__ void pix_split(int64_t p, int hw, int w, float inv_hw, float inv_w,
                                          int64_t &base, int &y, int &x) {
    {
        const int pi = (int)p;
        int b = (int)(((float)pi + 0.5f) * inv_hw);
        int rest = pi - b * hw;
        if (rest < 0) { --b; rest += hw; } else if (rest >= hw) { ++b; rest -= hw; }
        int yy = (int)(((float)rest + 0.5f) * inv_w);
        int xx = rest - yy * w;
        if (xx < 0) { --yy; xx += w; } else if (xx >= w) { ++yy; xx -= w; }
        base = (int64_t)b * hw;
        y = yy;
        x = xx;
    }
}

// kKB consecutive 16-wide k blocks per wave share its dout loads (9 cin / 16 is a
// multiple of 9, so of kKB).
constexpr int kKB = 3;

__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(
    const float *__restrict__ in, const float *__restrict__ dout, float *__restrict__ dw,
    float *__restrict__ dbias, int B, int H, int W, int cin, int cout, int chunk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npix = (int64_t)B * H * W;
    const int64_t pc = ((int64_t)blockIdx.x * 4 + wave) * chunk;   // past npix: an empty chunk
    const int kgroups = 9 * cin / (16 * kKB);
    const int kg = blockIdx.y % kgroups, cb2 = blockIdx.y / kgroups;
    int tap[kKB], c0[kKB], dy[kKB], dx[kKB];
#pragma unroll
    for (int q = 0; q < kKB; ++q) {
        const int kb = kg * kKB + q;
        tap[q] = (kb * 16) / cin;
        c0[q] = kb * 16 - tap[q] * cin;
        dy[q] = tap[q] / 3 - 1;
        dx[q] = tap[q] % 3 - 1;
    }
    const int co0 = cb2 * 32;
    const int r = lane & 15, g = lane >> 4;
    const int hw = H * W;
    const float inv_hw = 1.f / (float)hw, inv_w = 1.f / (float)W;
    v4f acc[kKB][2];
#pragma unroll
    for (int q = 0; q < kKB; ++q) acc[q][0] = acc[q][1] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bsum0 = 0.f, bsum1 = 0.f;
    const int64_t pend = pc + chunk < npix ? pc + chunk : npix;
    for (int64_t ps = pc; ps < pend; ps += 32) {
        // two steps of 16 pixels; this lane's four pixels of step h: ps + 16 h + 4 g + j
        float av0[2][4], av1[2][4], bv[2][kKB][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int64_t base;
            int y, x;
            pix_split(ps + 16 * h + 4 * g, hw, W, inv_hw, inv_w, base, y, x);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t p = ps + 16 * h + 4 * g + j;
                const bool live = p < pend;
                av0[h][j] = live ? dout[p * cout + co0 + r] : 0.f;
                av1[h][j] = live ? dout[p * cout + co0 + 16 + r] : 0.f;
#pragma unroll
                for (int q = 0; q < kKB; ++q) {
                    const int yy = y + dy[q], xx = x + dx[q];
                    bv[h][q][j] = (live && yy >= 0 && yy < H && xx >= 0 && xx < W)
                                      ? in[(base + (int64_t)yy * W + xx) * cin + c0[q] + r] : 0.f;
                }
                // next pixel in raster order
                if (++x == W) {
                    x = 0;
                    if (++y == H) {
                        y = 0;
                        base += hw;
                    }
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bsum0 += av0[h][0] + av0[h][1] + av0[h][2] + av0[h][3];
            bsum1 += av1[h][0] + av1[h][1] + av1[h][2] + av1[h][3];
            const v4s a0 = bf16x4(make_float4(av0[h][0], av0[h][1], av0[h][2], av0[h][3]));
            const v4s a1 = bf16x4(make_float4(av1[h][0], av1[h][1], av1[h][2], av1[h][3]));
#pragma unroll
            for (int q = 0; q < kKB; ++q) {
                const v4s b = bf16x4(make_float4(bv[h][q][0], bv[h][q][1], bv[h][q][2], bv[h][q][3]));
                acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[q][0], 0, 0, 0);
                acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, acc[q][1], 0, 0, 0);
            }
        }
    }
    // the four waves' blocks are summed in LDS, then one set of atomics per workgroup
    // (a quarter of the dw atomics of one set per wave)
    __shared__ float red[4][kKB * 8 + 2][64];
#pragma unroll
    for (int q = 0; q < kKB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            red[wave][q * 8 + i][lane] = acc[q][0][i];
            red[wave][q * 8 + 4 + i][lane] = acc[q][1][i];
        }
    red[wave][kKB * 8][lane] = bsum0;
    red[wave][kKB * 8 + 1][lane] = bsum1;
    __syncthreads();
    // accumulator rows are output channels 4 g + i, column k = c0 + r of the block's tap;
    // thread t sums entry (v, l) = (t / 64 + 4 m, t % 64) over the waves
    const int kin = 9 * cin;
    for (int v = wave; v < kKB * 8; v += 4) {
        const float sum = red[0][v][lane] + red[1][v][lane] + red[2][v][lane] + red[3][v][lane];
        const int q = v >> 3, cb = (v >> 2) & 1, i = v & 3;
        atomicAdd(&dw[(size_t)(co0 + cb * 16 + g * 4 + i) * kin + tap[q] * cin + c0[q] + r], sum);
    }
    if (dbias && kg == 0 && wave < 2) {
        // bias gradient from the same dout values (FP32, not rounded): sum the waves,
        // then the four pixel groups of each output channel
        const int v = kKB * 8 + wave;
        float bs = red[0][v][lane] + red[1][v][lane] + red[2][v][lane] + red[3][v][lane];
        bs += __shfl_xor(bs, 16);
        bs += __shfl_xor(bs, 32);
        if (g == 0) atomicAdd(&dbias[co0 + wave * 16 + r], bs);
    }
}

// ---- weight gradient, LDS-staged ----------------------------------------------
// For layers whose input channels come in multiples of 32.  A workgroup owns a
// 32 (cout) x 32 (cin) x 9 (tap) block of dw and a run of 8 x 32-pixel tiles.  Per
// tile it stages dout ([cout][row][column], BF16) and the input rows y0-1 .. y0+8,
// columns x0-1 .. x0+32 ([cin][row][column], BF16) in LDS -- every value fetched
// once per tile instead of once per tap -- and each wave (16 couts x 16 cins, the
// nine taps in 9 accumulators) contracts over the tile's rows, 32 pixels per
// v_mfma_f32_16x16x32_bf16: a lane takes 8 consecutive pixels of a row, its dout
// values one aligned 16-byte read, its input values for the three column taps one
// aligned 16-byte read and two neighbours shifted in (v_alignbit), so the taps
// share their loads.  The block goes to dw (and the bias gradient, from the blocks
// of the first 32 input channels) with FP32 atomics.  Runs of tiles are sized for
// about 512 workgroups: more would add dw atomics faster than they add parallelism
// (512^2 pixels, 32 -> 32 channels: 0.066 ms with one tile per workgroup, 0.046 ms
// with two; a 64^2 layer, 256 -> 256: 0.038 ms at 768 workgroups, 0.029 at 512).
constexpr int kWgTH = 8;                                // tile rows: the contraction's 32-pixel steps
constexpr int kWgDPitch = kWgTH * 32 + 8;               // dout tile, per output channel (elements)
constexpr int kWgXCols = 48;                            // input halo columns x0 - 8 .. x0 + 39
constexpr int kWgXPitch = (kWgTH + 2) * kWgXCols + 8;   // input halo, per input channel (elements)
constexpr int64_t kWgradWorkgroups = 512;
constexpr int64_t kWgradMaxRun = 64;

__global__ __launch_bounds__(256) void conv3x3_wgrad_lds_kernel(
    const float *__restrict__ in, const float *__restrict__ dout, float *__restrict__ dw,
    float *__restrict__ dbias, int H, int W, int cin, int cout, int tiles_x, int tiles_y, int64_t ntiles,
    int run) {
    __shared__ __align__(16) uint16_t dT[32 * kWgDPitch];
    __shared__ __align__(16) uint16_t xT[32 * kWgXPitch];
    __shared__ float bred[4][8][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int cbn = cout / 32;
    const int cb = blockIdx.y % cbn, cib = blockIdx.y / cbn;
    const int co0 = cb * 32, ci0 = cib * 32;
    const int wco = wave >> 1, wci = wave & 1;
    const bool want_bias = dbias && cib == 0;
    v4f acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bs[4] = {0.f, 0.f, 0.f, 0.f};
    const int64_t t0 = (int64_t)blockIdx.x * run;   // this workgroup's run of tiles
    const int64_t t1 = t0 + run < ntiles ? t0 + run : ntiles;
    for (int64_t t = t0; t < t1; ++t) {
        const int tx = (int)(t % tiles_x);
        const int64_t rest = t / tiles_x;
        const int ty = (int)(rest % tiles_y);
        const int64_t b = rest / tiles_y;
        const int y0 = ty * kWgTH, x0 = tx * 32;
        const size_t img = (size_t)b * H * W;
        __syncthreads();   // the previous tile has been read
        // dout tile, transposed to [channel][row][column] (BF16); zero past the image
        for (int i = tid; i < kWgTH * 32 * 8; i += 256) {
            const int q = i & 7, pix = i >> 3;
            const int rr = pix >> 5, cc = pix & 31;
            const int y = y0 + rr, x = x0 + cc;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (y < H && x < W) v = *reinterpret_cast<const float4 *>(dout + (img + (size_t)y * W + x) * cout + co0 + 4 * q);
            bs[0] += v.x; bs[1] += v.y; bs[2] += v.z; bs[3] += v.w;
            const v4s h = bf16x4(v);
            uint16_t *d = dT + (4 * q) * kWgDPitch + rr * 32 + cc;
            d[0] = (uint16_t)h[0];
            d[kWgDPitch] = (uint16_t)h[1];
            d[2 * kWgDPitch] = (uint16_t)h[2];
            d[3 * kWgDPitch] = (uint16_t)h[3];
        }
        // input rows y0 - 1 .. y0 + kWgTH, columns x0 - 1 .. x0 + 32 (halo column index c + 7
        // holds x0 - 1 + c), transposed to [channel][row][column]; zero outside the image
        for (int i = tid; i < (kWgTH + 2) * 34 * 8; i += 256) {
            const int q = i & 7, pix = i >> 3;
            const int hr = pix / 34, hc = pix - hr * 34;
            const int y = y0 - 1 + hr, x = x0 - 1 + hc;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (y >= 0 && y < H && x >= 0 && x < W)
                v = *reinterpret_cast<const float4 *>(in + (img + (size_t)y * W + x) * cin + ci0 + 4 * q);
            const v4s h = bf16x4(v);
            uint16_t *d = xT + (4 * q) * kWgXPitch + hr * kWgXCols + hc + 7;
            d[0] = (uint16_t)h[0];
            d[kWgXPitch] = (uint16_t)h[1];
            d[2 * kWgXPitch] = (uint16_t)h[2];
            d[3 * kWgXPitch] = (uint16_t)h[3];
        }
        __syncthreads();
        // row r of the tile is one 32-pixel step: lane (g, r16) takes pixels 8 g .. 8 g + 7
        // of it, output channel r16 of the wave's 16 (A) and input channel r16 of its 16 (B)
        const uint16_t *arow = dT + (16 * wco + r16) * kWgDPitch + 8 * g;
        const uint16_t *xrow = xT + (16 * wci + r16) * kWgXPitch + 8 * g;
#pragma unroll 2
        for (int r = 0; r < kWgTH; ++r) {
            const v8bf a = *reinterpret_cast<const v8bf *>(arow + r * 32);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const uint16_t *xr = xrow + (r + dy) * kWgXCols;
                // columns 8 g + dx - 1 + i for dx = 0, 1, 2: the aligned 8 at 8 g + 8, and the
                // neighbours at 8 g + 7 and 8 g + 16 shifted in
                const uint4 c = *reinterpret_cast<const uint4 *>(xr + 8);
                const unsigned lo = (unsigned)xr[7] << 16, hi = xr[16];
                const uint4 c0 = make_uint4(__builtin_amdgcn_alignbit(c.x, lo, 16), __builtin_amdgcn_alignbit(c.y, c.x, 16),
                                            __builtin_amdgcn_alignbit(c.z, c.y, 16), __builtin_amdgcn_alignbit(c.w, c.z, 16));
                const uint4 c2 = make_uint4(__builtin_amdgcn_alignbit(c.y, c.x, 16), __builtin_amdgcn_alignbit(c.z, c.y, 16),
                                            __builtin_amdgcn_alignbit(c.w, c.z, 16), __builtin_amdgcn_alignbit(hi, c.w, 16));
                acc[3 * dy + 0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, c0), acc[3 * dy + 0], 0, 0, 0);
                acc[3 * dy + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, c), acc[3 * dy + 1], 0, 0, 0);
                acc[3 * dy + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, c2), acc[3 * dy + 2], 0, 0, 0);
            }
        }
    }
    // accumulator rows are output channels 4 g + i of the wave's 16, column r16 its input channel
    const int kin = 9 * cin;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            atomicAdd(&dw[(size_t)(co0 + 16 * wco + 4 * g + i) * kin + tap * cin + ci0 + 16 * wci + r16], acc[tap][i]);
    if (want_bias) {
        // thread tid staged output channels 4 (tid & 7) .. + 3 (FP32, not rounded)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = bs[e];
            v += __shfl_xor(v, 8);
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            bs[e] = v;
        }
        if (lane < 8)
#pragma unroll
            for (int e = 0; e < 4; ++e) bred[wave][lane][e] = bs[e];
        __syncthreads();
        if (tid < 32) {
            const int q = tid >> 2, e = tid & 3;
            atomicAdd(&dbias[co0 + 4 * q + e], bred[0][q][e] + bred[1][q][e] + bred[2][q][e] + bred[3][q][e]);
        }
    }
}

__global__ void flip_weights_kernel(const uint16_t *__restrict__ w, uint16_t *__restrict__ wt, int cin,
                                    int cout) {
    const int64_t n = (int64_t)cout * 9 * cin;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // i indexes wt[ci][tap][co]
        const int co = (int)(i % cout);
        const int64_t rest = i / cout;
        const int tap = (int)(rest % 9), ci = (int)(rest / 9);
        wt[i] = w[((int64_t)co * 9 + (8 - tap)) * cin + ci];
    }
}

__global__ void relu_backward_kernel(const float *__restrict__ y, const float *__restrict__ dy,
                                     float *__restrict__ dx, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dx[i] = y[i] > 0.f ? dy[i] : 0.f;
}

__global__ void pool2_kernel(const float *__restrict__ in, float *__restrict__ out, int B, int H, int W, int C,
                             int backward) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n = (int64_t)B * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int xo = (int)(t % Wo);
        t /= Wo;
        const int yo = (int)(t % Ho);
        const int64_t b = t / Ho;
        const int64_t base = ((b * H + 2 * yo) * W + 2 * xo) * C + c;
        const int64_t rowc = (int64_t)W * C;
        if (!backward) {
            out[i] = 0.25f * (in[base] + in[base + C] + in[base + rowc] + in[base + rowc + C]);
        } else {
            // in = dout [B][Ho][Wo][C], out = din [B][H][W][C]
            const float gq = 0.25f * in[i];
            out[base] = gq;
            out[base + C] = gq;
            out[base + rowc] = gq;
            out[base + rowc + C] = gq;
        }
    }
}

__global__ void up2_kernel(const float *__restrict__ in, float *__restrict__ out, int B, int H, int W, int C,
                           int backward) {
    // H, W: the small side
    const int64_t n = (int64_t)B * H * W * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int x = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int64_t b = t / H;
        const int64_t W2 = 2 * W;
        const int64_t base = ((b * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
        const int64_t rowc = W2 * C;
        if (!backward) {
            const float v = in[i];
            out[base] = v;
            out[base + C] = v;
            out[base + rowc] = v;
            out[base + rowc + C] = v;
        } else {
            // in = dout [B][2H][2W][C], out = din [B][H][W][C]
            out[i] = in[base] + in[base + C] + in[base + rowc] + in[base + rowc + C];
        }
    }
}

// Four channels per thread (float4) and 32-bit index arithmetic: the fast forms of
// pool2 / up2 / copy_channels for channel counts (and offsets) in multiples of 4
// and fewer than 2^31 work items, which the host checks.  A flat index split by
// 64-bit division costs dozens of instructions per element, more than the copy.
__global__ void pool2_v4_kernel(const float4 *__restrict__ in, float4 *__restrict__ out, int B, int H, int W, int q4,
                                int backward) {
    const unsigned Ho = (unsigned)H / 2, Wo = (unsigned)W / 2, q = (unsigned)q4;
    const unsigned n = (unsigned)B * Ho * Wo * q;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned c = i % q, t = i / q;
        const unsigned xo = t % Wo, t2 = t / Wo;
        const unsigned yo = t2 % Ho, b = t2 / Ho;
        const size_t base = (((size_t)b * H + 2 * yo) * W + 2 * xo) * q + c;
        const size_t rowc = (size_t)W * q;
        if (!backward) {
            const float4 a = in[base], bb = in[base + q], cc = in[base + rowc], d = in[base + rowc + q];
            out[i] = make_float4(0.25f * (a.x + bb.x + cc.x + d.x), 0.25f * (a.y + bb.y + cc.y + d.y),
                                 0.25f * (a.z + bb.z + cc.z + d.z), 0.25f * (a.w + bb.w + cc.w + d.w));
        } else {
            const float4 g = in[i];
            const float4 gq = make_float4(0.25f * g.x, 0.25f * g.y, 0.25f * g.z, 0.25f * g.w);
            out[base] = gq;
            out[base + q] = gq;
            out[base + rowc] = gq;
            out[base + rowc + q] = gq;
        }
    }
}

__global__ void up2_v4_kernel(const float4 *__restrict__ in, float4 *__restrict__ out, int B, int H, int W, int q4,
                              int backward) {
    // H, W: the small side
    const unsigned q = (unsigned)q4;
    const unsigned n = (unsigned)B * (unsigned)H * (unsigned)W * q;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned c = i % q, t = i / q;
        const unsigned x = t % (unsigned)W, t2 = t / (unsigned)W;
        const unsigned y = t2 % (unsigned)H, b = t2 / (unsigned)H;
        const size_t W2 = 2 * (size_t)W;
        const size_t base = (((size_t)b * 2 * H + 2 * y) * W2 + 2 * x) * q + c;
        const size_t rowc = W2 * q;
        if (!backward) {
            const float4 v = in[i];
            out[base] = v;
            out[base + q] = v;
            out[base + rowc] = v;
            out[base + rowc + q] = v;
        } else {
            const float4 a = in[base], bb = in[base + q], cc = in[base + rowc], d = in[base + rowc + q];
            out[i] = make_float4(a.x + bb.x + cc.x + d.x, a.y + bb.y + cc.y + d.y, a.z + bb.z + cc.z + d.z,
                                 a.w + bb.w + cc.w + d.w);
        }
    }
}

__global__ void copy_channels_v4_kernel(const float4 *__restrict__ src, int src_q, int src_off_q,
                                        float4 *__restrict__ dst, int dst_q, int dst_off_q, int count_q,
                                        unsigned n) {
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned p = i / (unsigned)count_q, c = i - p * (unsigned)count_q;
        dst[(size_t)p * dst_q + dst_off_q + c] = src[(size_t)p * src_q + src_off_q + c];
    }
}

__global__ void copy_channels_kernel(const float *__restrict__ src, int src_c, int src_off, float *__restrict__ dst,
                                     int dst_c, int dst_off, int count, int64_t npix) {
    const int64_t n = npix * count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / count;
        const int c = (int)(i - p * count);
        dst[p * dst_c + dst_off + c] = src[p * src_c + src_off + c];
    }
}

__global__ void axpy_kernel(const float *__restrict__ x, float *__restrict__ y, float a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ pb, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = (uint16_t)bf16(pi);
    }
}

inline int grid_for(int64_t n) {
    const int64_t blocks = (n + 255) / 256;
    return (int)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536);
}

inline int done(hipError_t e) { return e == hipSuccess ? 0 : -1; }

// the float4 kernels: channels in multiples of 4, 16-byte aligned tensors and work
// items that index in 31 bits
inline bool aligned16(const void *a, const void *b) {
    return (((uintptr_t)a | (uintptr_t)b) & 15) == 0;
}
inline bool fits_v4(int c, int64_t items) { return (c & 3) == 0 && items > 0 && items < ((int64_t)1 << 31); }

// 32-channel-slice convolution in 8-, 4- or 2-row tiles (the most rows that still
// give kConvWorkgroupsWanted workgroups, else 2)
void launch_tiled32(const ConvInput &src, const uint16_t *w, const float *bias, float *out, int B, int H, int W,
                    int cin, int cout, int relu, hipStream_t st) {
    const int tiles_x = (W + kTW - 1) / kTW, cb = cout / 32;
    const int64_t t8 = (int64_t)B * tiles_x * ((H + 7) / 8), t4 = (int64_t)B * tiles_x * ((H + 3) / 4),
                  t2 = (int64_t)B * tiles_x * ((H + 1) / 2);
    if (t8 * cb >= kConvWorkgroupsWanted)
        hipLaunchKernelGGL(conv3x3_tiled32_kernel<8>, dim3((unsigned)t8, cb), dim3(256), 0, st, src, w, bias, out, H,
                           W, cin, cout, relu, tiles_x, (H + 7) / 8);
    else if (t4 * cb >= kConvWorkgroupsWanted)
        hipLaunchKernelGGL(conv3x3_tiled32_kernel<4>, dim3((unsigned)t4, cb), dim3(256), 0, st, src, w, bias, out, H,
                           W, cin, cout, relu, tiles_x, (H + 3) / 4);
    else
        hipLaunchKernelGGL(conv3x3_tiled32_kernel<2>, dim3((unsigned)t2, cb), dim3(256), 0, st, src, w, bias, out, H,
                           W, cin, cout, relu, tiles_x, (H + 1) / 2);
}

}  // namespace


extern "C" {

int asf_warm_conv3x3(const float *in, const uint16_t *w, const float *bias, float *out, int32_t B, int32_t H,
                     int32_t W, int32_t cin, int32_t cout, int32_t relu, void *stream) {
    if (!in || !w || !out || B <= 0 || H <= 0 || W <= 0 || cin <= 0 || cout <= 0 || cin % 16 || cout % 32)
        return -1;
    const int64_t npix = (int64_t)B * H * W;
    // LDS-tiled unless the layer has fewer than 64 of its 8 x 32 tiles (times the
    // channel blocks); such small layers take the direct kernel's 16-pixel wave
    // tiles.  (Measured at 64^2 pixels, 256 -> 256 channels, 128 workgroups:
    // 0.054 ms tiled against 0.095 ms direct.)
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
    const int64_t tiles = (int64_t)B * tiles_x * tiles_y;
    if (tiles * (cout / 32) >= 64 && tiles < (int64_t)1 << 31) {
        const int cb = cout / 32;
        if (cin % 32 == 0) {
            hipStream_t st = static_cast<hipStream_t>(stream);
            launch_tiled32(ConvInput{in, nullptr, nullptr, 0}, w, bias, out, B, H, W, cin, cout, relu, st);
        } else {
            hipLaunchKernelGGL(conv3x3_tiled_kernel, dim3((unsigned)tiles, cb), dim3(256), 0,
                               static_cast<hipStream_t>(stream), in, w, bias, out, H, W, cin, cout, relu, tiles_x,
                               tiles_y);
        }
    } else {
        const int64_t tiles16 = (npix + 15) / 16;
        const dim3 grid((unsigned)((tiles16 + kConvWaves - 1) / kConvWaves), (unsigned)(cout / 32));
        hipLaunchKernelGGL(conv3x3_kernel<1>, grid, dim3(64 * kConvWaves), 0, static_cast<hipStream_t>(stream), in,
                           w, bias, out, B, H, W, cin, cout, relu);
    }
    return done(hipGetLastError());
}

int asf_warm_conv3x3_upcat(const float *low, int32_t c_low, const float *skip, int32_t c_skip, const uint16_t *w,
                           const float *bias, float *out, int32_t B, int32_t H, int32_t W, int32_t cout,
                           int32_t relu, void *stream) {
    if (!low || !skip || !w || !out || B <= 0 || H <= 1 || W <= 1 || (H & 1) || (W & 1) || c_low <= 0 ||
        c_skip <= 0 || c_low % 32 || c_skip % 32 || cout <= 0 || cout % 32)
        return -1;
    const int64_t tiles = (int64_t)B * ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
    if (tiles * (cout / 32) < 64 || tiles >= ((int64_t)1 << 30)) return -1;   // the tiled layers only
    launch_tiled32(ConvInput{nullptr, low, skip, c_low}, w, bias, out, B, H, W, c_low + c_skip, cout, relu,
                   static_cast<hipStream_t>(stream));
    return done(hipGetLastError());
}

int asf_warm_conv3x3_wgrad(const float *in, const float *dout, float *dw, float *dbias, int32_t B, int32_t H,
                           int32_t W, int32_t cin, int32_t cout, void *stream) {
    if (!in || !dout || !dw || B <= 0 || H <= 0 || W <= 0 || cin <= 0 || cout <= 0 || cin % 16 || cout % 32)
        return -1;
    const int64_t npix = (int64_t)B * H * W;
    if (npix >= kMaxWgradPix) return -1;
    if (cin % 32 == 0) {
        const int tiles_x = (W + 31) / 32, tiles_y = (H + kWgTH - 1) / kWgTH;
        const int64_t ntiles = (int64_t)B * tiles_x * tiles_y;
        const int64_t blocks = (int64_t)(cout / 32) * (cin / 32);
        int64_t run = ntiles * blocks / kWgradWorkgroups;   // tiles per workgroup
        if (run < 1) run = 1;
        if (run > kWgradMaxRun) run = kWgradMaxRun;
        const dim3 grid((unsigned)((ntiles + run - 1) / run), (unsigned)blocks);
        hipLaunchKernelGGL(conv3x3_wgrad_lds_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), in, dout,
                           dw, dbias, H, W, cin, cout, tiles_x, tiles_y, ntiles, (int)run);
        return done(hipGetLastError());
    }
    // the longer chunk where it still leaves at least 1024 workgroups
    const int64_t kgroups = 9 * cin / (16 * kKB);
    const int64_t wg_large = (npix + 4 * kWgradChunkLarge - 1) / (4 * kWgradChunkLarge) * (cout / 32) * kgroups;
    const int chunk = wg_large >= 1024 ? kWgradChunkLarge : kWgradChunkSmall;
    const int64_t chunks = (npix + chunk - 1) / chunk;
    const dim3 grid((unsigned)((chunks + 3) / 4), (unsigned)((cout / 32) * (9 * cin / (16 * kKB))));
    hipLaunchKernelGGL(conv3x3_wgrad_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), in, dout, dw,
                       dbias, B, H, W, cin, cout, chunk);
    return done(hipGetLastError());
}

int asf_warm_flip_weights(const uint16_t *w, uint16_t *wt, int32_t cin, int32_t cout, void *stream) {
    if (!w || !wt || cin <= 0 || cout <= 0) return -1;
    hipLaunchKernelGGL(flip_weights_kernel, dim3(grid_for((int64_t)cout * 9 * cin)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), w, wt, cin, cout);
    return done(hipGetLastError());
}

int asf_warm_relu_backward(const float *y, const float *dy, float *dx, int64_t n, void *stream) {
    if (!y || !dy || !dx || n <= 0) return -1;
    hipLaunchKernelGGL(relu_backward_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), y,
                       dy, dx, n);
    return done(hipGetLastError());
}

int asf_warm_pool2(const float *in, float *out, int32_t B, int32_t H, int32_t W, int32_t C, void *stream) {
    if (!in || !out || B <= 0 || H <= 1 || W <= 1 || C <= 0 || (H & 1) || (W & 1)) return -1;
    if (fits_v4(C, (int64_t)B * (H / 2) * (W / 2) * (C / 4)) && aligned16(in, out)) {
        hipLaunchKernelGGL(pool2_v4_kernel, dim3(grid_for((int64_t)B * (H / 2) * (W / 2) * (C / 4))), dim3(256), 0,
                           static_cast<hipStream_t>(stream), reinterpret_cast<const float4 *>(in),
                           reinterpret_cast<float4 *>(out), B, H, W, C / 4, 0);
        return done(hipGetLastError());
    }
    hipLaunchKernelGGL(pool2_kernel, dim3(grid_for((int64_t)B * H * W * C / 4)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), in, out, B, H, W, C, 0);
    return done(hipGetLastError());
}

int asf_warm_pool2_backward(const float *dout, float *din, int32_t B, int32_t H, int32_t W, int32_t C,
                            void *stream) {
    if (!dout || !din || B <= 0 || H <= 1 || W <= 1 || C <= 0 || (H & 1) || (W & 1)) return -1;
    if (fits_v4(C, (int64_t)B * (H / 2) * (W / 2) * (C / 4)) && aligned16(dout, din)) {
        hipLaunchKernelGGL(pool2_v4_kernel, dim3(grid_for((int64_t)B * (H / 2) * (W / 2) * (C / 4))), dim3(256), 0,
                           static_cast<hipStream_t>(stream), reinterpret_cast<const float4 *>(dout),
                           reinterpret_cast<float4 *>(din), B, H, W, C / 4, 1);
        return done(hipGetLastError());
    }
    hipLaunchKernelGGL(pool2_kernel, dim3(grid_for((int64_t)B * H * W * C / 4)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dout, din, B, H, W, C, 1);
    return done(hipGetLastError());
}

int asf_warm_up2(const float *in, float *out, int32_t B, int32_t H, int32_t W, int32_t C, void *stream) {
    if (!in || !out || B <= 0 || H <= 0 || W <= 0 || C <= 0) return -1;
    if (fits_v4(C, (int64_t)B * H * W * (C / 4)) && aligned16(in, out)) {
        hipLaunchKernelGGL(up2_v4_kernel, dim3(grid_for((int64_t)B * H * W * (C / 4))), dim3(256), 0,
                           static_cast<hipStream_t>(stream), reinterpret_cast<const float4 *>(in),
                           reinterpret_cast<float4 *>(out), B, H, W, C / 4, 0);
        return done(hipGetLastError());
    }
    hipLaunchKernelGGL(up2_kernel, dim3(grid_for((int64_t)B * H * W * C)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), in, out, B, H, W, C, 0);
    return done(hipGetLastError());
}

int asf_warm_up2_backward(const float *dout, float *din, int32_t B, int32_t H, int32_t W, int32_t C,
                          void *stream) {
    if (!dout || !din || B <= 0 || H <= 0 || W <= 0 || C <= 0) return -1;
    if (fits_v4(C, (int64_t)B * H * W * (C / 4)) && aligned16(dout, din)) {
        hipLaunchKernelGGL(up2_v4_kernel, dim3(grid_for((int64_t)B * H * W * (C / 4))), dim3(256), 0,
                           static_cast<hipStream_t>(stream), reinterpret_cast<const float4 *>(dout),
                           reinterpret_cast<float4 *>(din), B, H, W, C / 4, 1);
        return done(hipGetLastError());
    }
    hipLaunchKernelGGL(up2_kernel, dim3(grid_for((int64_t)B * H * W * C)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dout, din, B, H, W, C, 1);
    return done(hipGetLastError());
}

int asf_warm_copy_channels(const float *src, int32_t src_c, int32_t src_off, float *dst, int32_t dst_c,
                           int32_t dst_off, int32_t count, int64_t npix, void *stream) {
    if (!src || !dst || count <= 0 || npix <= 0 || src_off < 0 || dst_off < 0 || src_off + count > src_c ||
        dst_off + count > dst_c)
        return -1;
    if (((src_c | src_off | dst_c | dst_off | count) & 3) == 0 && fits_v4(4, npix * (count / 4)) && aligned16(src, dst)) {
        const int64_t n = npix * (count / 4);
        hipLaunchKernelGGL(copy_channels_v4_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                           reinterpret_cast<const float4 *>(src), src_c / 4, src_off / 4,
                           reinterpret_cast<float4 *>(dst), dst_c / 4, dst_off / 4, count / 4, (unsigned)n);
        return done(hipGetLastError());
    }
    hipLaunchKernelGGL(copy_channels_kernel, dim3(grid_for(npix * count)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), src, src_c, src_off, dst, dst_c, dst_off, count, npix);
    return done(hipGetLastError());
}

int asf_warm_axpy(const float *x, float *y, float a, int64_t n, void *stream) {
    if (!x || !y || n <= 0) return -1;
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, y, a, n);
    return done(hipGetLastError());
}

int asf_warm_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, float b1,
                  float b2, float eps, int32_t t, void *stream) {
    if (!p || !g || !m || !v || n <= 0 || t < 1) return -1;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g, m, v,
                       pb, n, lr, b1, b2, eps, c1, c2);
    return done(hipGetLastError());
}

}  // extern "C"
