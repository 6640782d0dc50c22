/*
 * asf_warm.h -- C ABI of the kernels behind the learned warm start for
 * phase-hologram descent on a curved surface (the gradient-based synthesis that
 * the adjoint of Eq. (7)-(9) enables): a small convolutional encoder-decoder
 * that maps a target intensity and the surface height to a source phase.
 *
 * Tensors are DEVICE pointers, caller-owned, channels-last ("NHWC"): element
 * (b, y, x, c) of a [B][H][W][C] tensor sits at ((b H + y) W + x) C + c.
 * Activations and gradients are FP32; convolution weights are BF16 (raw 16-bit
 * patterns, round-to-nearest-even from FP32) laid out [Cout][3][3][Cin]
 * (k = (ky 3 + kx) Cin + ci fastest); products run on the matrix cores
 * (BF16 x BF16 -> FP32 accumulation).  Streams are hipStream_t as void*.
 * Every function is asynchronous and returns 0, or -1 for an invalid argument
 * (null pointer, a size <= 0, or a channel count the kernel does not take).
 */
#ifndef ASF_WARM_H
#define ASF_WARM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * 3x3 convolution, stride 1, zero padding 1:
 *   out[b,y,x,co] = bias[co] + sum_{ky,kx,ci} in[b, y+ky-1, x+kx-1, ci] w[co, ky, kx, ci]
 * then max(0, .) if relu.  in [B][H][W][cin] FP32 (rounded to BF16 on load),
 * w [cout][3][3][cin] BF16, bias [cout] FP32 or NULL, out [B][H][W][cout] FP32.
 * cin a multiple of 16, cout a multiple of 32.
 */
int asf_warm_conv3x3(const float *in, const uint16_t *w, const float *bias, float *out, int32_t B,
                     int32_t H, int32_t W, int32_t cin, int32_t cout, int32_t relu, void *stream);

/*
 * asf_warm_conv3x3 of the decoder's concatenated input, read in place: channels
 * 0 .. c_low-1 are the 2x nearest-neighbour upsampling of low [B][H/2][W/2][c_low],
 * channels c_low .. c_low+c_skip-1 are skip [B][H][W][c_skip]; w [cout][3][3][c_low+c_skip].
 * The result equals (bit for bit) asf_warm_up2 and two asf_warm_copy_channels into
 * one tensor followed by asf_warm_conv3x3.  H, W even; c_low, c_skip multiples of 32,
 * cout a multiple of 32; layers with fewer than 64 (8 x 32-pixel tiles x cout/32)
 * are refused (-1): the caller concatenates those.
 */
int asf_warm_conv3x3_upcat(const float *low, int32_t c_low, const float *skip, int32_t c_skip,
                           const uint16_t *w, const float *bias, float *out, int32_t B, int32_t H,
                           int32_t W, int32_t cout, int32_t relu, void *stream);

/*
 * Weight gradient of asf_warm_conv3x3 (before the activation):
 *   dw[co, ky, kx, ci] += sum_{b,y,x} dout[b,y,x,co] in[b, y+ky-1, x+kx-1, ci]
 *   dbias[co] += sum_{b,y,x} dout[b,y,x,co]      (dbias may be NULL)
 * in and dout rounded to BF16 on load, FP32 products summed with FP32 atomics
 * (accumulates: clear dw and dbias first).  dw [cout][3][3][cin] FP32.
 * B H W must be below 2^22 (-1 otherwise).
 */
int asf_warm_conv3x3_wgrad(const float *in, const float *dout, float *dw, float *dbias, int32_t B,
                           int32_t H, int32_t W, int32_t cin, int32_t cout, void *stream);

/*
 * Weights of the input gradient: wt[ci, ky, kx, co] = w[co, 2-ky, 2-kx, ci], so that
 * asf_warm_conv3x3(dout, wt, NULL, din, ..., cin = cout, cout = cin, relu = 0) is
 * the gradient with respect to the convolution's input.
 */
int asf_warm_flip_weights(const uint16_t *w, uint16_t *wt, int32_t cin, int32_t cout, void *stream);

/* dx[i] = dy[i] if y[i] > 0 else 0 (ReLU backward from the ReLU's output), n elements. */
int asf_warm_relu_backward(const float *y, const float *dy, float *dx, int64_t n, void *stream);

/* 2x2 average pooling [B][H][W][C] -> [B][H/2][W/2][C] (H, W even); and its gradient. */
int asf_warm_pool2(const float *in, float *out, int32_t B, int32_t H, int32_t W, int32_t C, void *stream);
int asf_warm_pool2_backward(const float *dout, float *din, int32_t B, int32_t H, int32_t W, int32_t C,
                            void *stream);

/* Nearest 2x upsampling [B][H][W][C] -> [B][2H][2W][C]; and its gradient (sum over each 2x2). */
int asf_warm_up2(const float *in, float *out, int32_t B, int32_t H, int32_t W, int32_t C, void *stream);
int asf_warm_up2_backward(const float *dout, float *din, int32_t B, int32_t H, int32_t W, int32_t C,
                          void *stream);

/*
 * Channel slice copy between channels-last tensors of npix pixels:
 *   dst[p, dst_off + c] = src[p, src_off + c] for c < count
 * (builds the decoder's concatenations and splits their gradients).
 */
int asf_warm_copy_channels(const float *src, int32_t src_c, int32_t src_off, float *dst, int32_t dst_c,
                           int32_t dst_off, int32_t count, int64_t npix, void *stream);

/* y[i] += a x[i], n elements (sums the gradients of a tensor used twice). */
int asf_warm_axpy(const float *x, float *y, float a, int64_t n, void *stream);

/*
 * One Adam step (Kingma and Ba) on n FP32 parameters with bias-corrected moments:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 * and the BF16 copy pb[i] = bf16(p[i]) if pb is not NULL.  t >= 1 is the step count.
 */
int asf_warm_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr,
                  float b1, float b2, float eps, int32_t t, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ASF_WARM_H */
