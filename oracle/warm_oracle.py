"""CPU oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.

A plain FP64 numpy statement of what the GPU kernels of include/asf_warm.h
compute: 3x3 convolutions (stride 1, zero padding 1) with bias and ReLU, their
weight and input gradients, 2x2 average pooling, nearest 2x upsampling, channel
concatenation, and the encoder-decoder built from them, forward and backward.

Tensors are channels-last, (B, H, W, C); weights (Cout, 3, 3, Cin).  The GPU
multiplies BF16 operands with FP32 accumulation; with ``rounded=True`` the
oracle takes the same precision decision -- every operand of a convolution
product is rounded to BF16 (round to nearest even, from its FP32 value) before
the exact FP64 product and sum -- so the two agree up to the order of the FP32
sums.  With ``rounded=False`` everything is exact FP64 (used to pin the
backward against finite differences).  Nothing here is shared with the GPU path.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to BF16 (nearest even) from FP32, returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _q(x, rounded):
    return bf16(x) if rounded else np.asarray(x, dtype=np.float64)


def _shifted(x, dy, dx):
    """x shifted so that out[b, y, x] = x[b, y + dy, x + dx] (zero outside)."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[:, ys:ye, xs:xe, :] = x[:, ys + dy:ye + dy, xs + dx:xe + dx, :]
    return out


def conv3x3(x, w, b=None, relu=False, rounded=True):
    """out[b,y,x,co] = bias[co] + sum_{ky,kx,ci} x[b,y+ky-1,x+kx-1,ci] w[co,ky,kx,ci]."""
    xq, wq = _q(x, rounded), _q(w, rounded)
    out = np.zeros(x.shape[:3] + (w.shape[0],))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("bhwc,oc->bhwo", _shifted(xq, ky - 1, kx - 1), wq[:, ky, kx, :])
    if b is not None:
        out += b
    return np.maximum(out, 0.0) if relu else out


def conv3x3_input_grad(dout, w, rounded=True):
    """d/dx of sum(dout * conv3x3(x, w)): a convolution with the flipped weights."""
    dq, wq = _q(dout, rounded), _q(w, rounded)
    dx = np.zeros(dout.shape[:3] + (w.shape[3],))
    for ky in range(3):
        for kx in range(3):
            # x[y'] feeds out[y' - (ky - 1)]
            dx += np.einsum("bhwo,oc->bhwc", _shifted(dq, 1 - ky, 1 - kx), wq[:, ky, kx, :])
    return dx


def conv3x3_weight_grad(x, dout, rounded=True):
    """(dw, dbias) of sum(dout * conv3x3(x, w, b)); dbias sums the unrounded dout."""
    xq, dq = _q(x, rounded), _q(dout, rounded)
    dw = np.zeros((dout.shape[3], 3, 3, x.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dq, _shifted(xq, ky - 1, kx - 1))
    return dw, np.asarray(dout, dtype=np.float64).sum(axis=(0, 1, 2))


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(d):
    return np.repeat(np.repeat(d, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(d):
    B, H2, W2, C = d.shape
    return d.reshape(B, H2 // 2, 2, W2 // 2, 2, C).sum(axis=(2, 4))


# ---------------------------------------------------------------------------
# the encoder-decoder: layer list (cin, cout, relu) for base width c and input
# channels cin0 (padded); four levels, skip connections by concatenation
# ---------------------------------------------------------------------------

def layer_shapes(c=32, cin0=16, cout_head=32):
    return [(cin0, c, True), (c, c, True),
            (c, 2 * c, True), (2 * c, 2 * c, True),
            (2 * c, 4 * c, True), (4 * c, 4 * c, True),
            (4 * c, 8 * c, True), (8 * c, 8 * c, True),
            (12 * c, 4 * c, True), (4 * c, 4 * c, True),
            (6 * c, 2 * c, True), (2 * c, 2 * c, True),
            (3 * c, c, True), (c, c, True),
            (c, cout_head, False)]


def net_forward(x, params, rounded=True):
    """Output (B, H, W, cout_head) and the cache for net_backward.  params: list of (w, b)."""
    conv = lambda t, i: conv3x3(t, params[i][0], params[i][1], relu=True, rounded=rounded)
    cache = {}
    a = [None] * 15
    a[0] = conv(x, 0); a[1] = conv(a[0], 1)
    p1 = pool2(a[1]); a[2] = conv(p1, 2); a[3] = conv(a[2], 3)
    p2 = pool2(a[3]); a[4] = conv(p2, 4); a[5] = conv(a[4], 5)
    p3 = pool2(a[5]); a[6] = conv(p3, 6); a[7] = conv(a[6], 7)
    c3 = np.concatenate([up2(a[7]), a[5]], axis=3); a[8] = conv(c3, 8); a[9] = conv(a[8], 9)
    c2 = np.concatenate([up2(a[9]), a[3]], axis=3); a[10] = conv(c2, 10); a[11] = conv(a[10], 11)
    c1 = np.concatenate([up2(a[11]), a[1]], axis=3); a[12] = conv(c1, 12); a[13] = conv(a[12], 13)
    a[14] = conv3x3(a[13], params[14][0], params[14][1], relu=False, rounded=rounded)
    cache.update(x=x, a=a, p1=p1, p2=p2, p3=p3, c3=c3, c2=c2, c1=c1)
    return a[14], cache


def net_backward(dout, params, cache, rounded=True):
    """Gradients [(dw, db)] of sum(dout * output) for every layer."""
    a = cache["a"]
    inputs = {0: cache["x"], 1: a[0], 2: cache["p1"], 3: a[2], 4: cache["p2"], 5: a[4], 6: cache["p3"],
              7: a[6], 8: cache["c3"], 9: a[8], 10: cache["c2"], 11: a[10], 12: cache["c1"], 13: a[12],
              14: a[13]}
    grads = [None] * 15

    def layer(i, dy, relu=True, need_input=True):
        dpre = np.where(a[i] > 0, dy, 0.0) if relu else dy
        grads[i] = conv3x3_weight_grad(inputs[i], dpre, rounded)
        return conv3x3_input_grad(dpre, params[i][0], rounded) if need_input else None

    d13 = layer(14, dout, relu=False)
    d12 = layer(13, d13)
    dc1 = layer(12, d12)
    c = a[11].shape[3]
    d11 = up2_backward(dc1[..., :c]); d1_skip = dc1[..., c:]
    d10 = layer(11, d11)
    dc2 = layer(10, d10)
    c = a[9].shape[3]
    d9 = up2_backward(dc2[..., :c]); d3_skip = dc2[..., c:]
    d8 = layer(9, d9)
    dc3 = layer(8, d8)
    c = a[7].shape[3]
    d7 = up2_backward(dc3[..., :c]); d5_skip = dc3[..., c:]
    d6 = layer(7, d7)
    dp3 = layer(6, d6)
    d5 = pool2_backward(dp3) + d5_skip
    d4 = layer(5, d5)
    dp2 = layer(4, d4)
    d3 = pool2_backward(dp2) + d3_skip
    d2 = layer(3, d3)
    dp1 = layer(2, d2)
    d1 = pool2_backward(dp1) + d1_skip
    d0 = layer(1, d1)
    layer(0, d0, need_input=False)
    return grads
