"""GPU kernels of the learned warm start against the FP64 oracle of the network
(oracle/warm_oracle.py), which rounds the convolution operands to BF16 exactly
where the kernels do; and the network's gradient end to end."""
import ctypes

import numpy as np
import pytest

from gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _setup():
    torch = torch_gpu()
    import paper_1203_3583_amd.warmstart as ws
    from oracle import warm_oracle as wo
    return torch, ws, wo


def _weights(torch, ws, rng, cout, cin, scale=0.2):
    w = (rng.standard_normal((cout, 9 * cin)) * scale).astype(np.float32)
    wt = torch.from_numpy(w).cuda()
    return wt, ws.bf16_bits(torch, wt), w.reshape(cout, 3, 3, cin)


# every kernel: direct with 16-pixel wave tiles (the three small cases), LDS-tiled with
# 16-channel slices (the next three: ragged tiles on both axes, several images) and with
# 32-channel slices in 8-, 4- and 2-row tiles (the last three, ragged as well)
@pytest.mark.parametrize("B,H,W,cin,cout,relu", [(2, 8, 12, 16, 32, True), (1, 5, 7, 48, 64, False),
                                                 (1, 16, 16, 32, 96, True), (1, 300, 250, 16, 32, False),
                                                 (2, 255, 259, 16, 64, True), (3, 203, 100, 48, 64, False),
                                                 (1, 517, 500, 32, 64, True), (2, 203, 257, 64, 64, False),
                                                 (1, 299, 250, 96, 32, True)])
def test_conv3x3_forward(B, H, W, cin, cout, relu):
    torch, ws, wo = _setup()
    rng = np.random.default_rng(B * 100 + cin)
    x = rng.standard_normal((B, H, W, cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    wt, wb, w4 = _weights(torch, ws, rng, cout, cin)
    xt, bt = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
    out = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    L = ws._lib()
    s = ws._stream(torch)
    assert L.asf_warm_conv3x3(ws._ptr(xt), ws._ptr(wb), ws._ptr(bt), ws._ptr(out), B, H, W, cin, cout,
                              int(relu), s) == 0
    want = wo.conv3x3(x, wo.bf16(w4), b, relu=relu)
    err = _rel(out.cpu().numpy(), want)
    print(f"conv {B}x{H}x{W} {cin}->{cout}: {err:.2e}")
    assert err < 1e-5
    # invalid channel counts are refused
    assert L.asf_warm_conv3x3(ws._ptr(xt), ws._ptr(wb), None, ws._ptr(out), B, H, W, cin + 1, cout, 0, s) == -1


# the decoder's concatenation read in place, in 8-, 4- and 2-row tiles (the last ragged and two
# images): bit for bit what upsampling, two channel copies and the convolution give
@pytest.mark.parametrize("B,H,W,c_low,c_skip,cout", [(1, 512, 512, 64, 32, 32), (1, 256, 256, 32, 64, 64),
                                                     (2, 130, 70, 32, 32, 64)])
def test_conv3x3_upcat_matches_concatenation(B, H, W, c_low, c_skip, cout):
    torch, ws, wo = _setup()
    rng = np.random.default_rng(H + c_low)
    low = torch.from_numpy(rng.standard_normal((B, H // 2, W // 2, c_low)).astype(np.float32)).cuda()
    skip = torch.from_numpy(rng.standard_normal((B, H, W, c_skip)).astype(np.float32)).cuda()
    cin = c_low + c_skip
    _, wb, _ = _weights(torch, ws, rng, cout, cin)
    bt = torch.from_numpy(rng.standard_normal(cout).astype(np.float32)).cuda()
    L = ws._lib()
    s = ws._stream(torch)
    fused = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    assert L.asf_warm_conv3x3_upcat(ws._ptr(low), c_low, ws._ptr(skip), c_skip, ws._ptr(wb), ws._ptr(bt),
                                    ws._ptr(fused), B, H, W, cout, 1, s) == 0
    up = torch.empty((B, H, W, c_low), dtype=torch.float32, device="cuda")
    assert L.asf_warm_up2(ws._ptr(low), ws._ptr(up), B, H // 2, W // 2, c_low, s) == 0
    cat = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    assert L.asf_warm_copy_channels(ws._ptr(up), c_low, 0, ws._ptr(cat), cin, 0, c_low, B * H * W, s) == 0
    assert L.asf_warm_copy_channels(ws._ptr(skip), c_skip, 0, ws._ptr(cat), cin, c_low, c_skip, B * H * W, s) == 0
    want = torch.empty_like(fused)
    assert L.asf_warm_conv3x3(ws._ptr(cat), ws._ptr(wb), ws._ptr(bt), ws._ptr(want), B, H, W, cin, cout, 1, s) == 0
    assert np.array_equal(fused.cpu().numpy(), want.cpu().numpy())
    # refused: odd size, channel counts off 32, a layer too small for the tiled kernel
    assert L.asf_warm_conv3x3_upcat(ws._ptr(low), c_low, ws._ptr(skip), c_skip, ws._ptr(wb), None,
                                    ws._ptr(fused), B, H - 1, W, cout, 0, s) == -1
    assert L.asf_warm_conv3x3_upcat(ws._ptr(low), c_low - 16, ws._ptr(skip), c_skip + 16, ws._ptr(wb), None,
                                    ws._ptr(fused), B, H, W, cout, 0, s) == -1
    assert L.asf_warm_conv3x3_upcat(ws._ptr(low), c_low, ws._ptr(skip), c_skip, ws._ptr(wb), None,
                                    ws._ptr(fused), 1, 16, 16, cout, 0, s) == -1


# direct kernel (16 and 48 input channels), LDS-staged kernel (multiples of 32: one tile per
# workgroup, then runs of tiles crossing image boundaries with one and two input-channel blocks)
@pytest.mark.parametrize("B,H,W,cin,cout", [(2, 8, 12, 16, 32), (1, 5, 7, 48, 64), (3, 32, 32, 32, 32),
                                            (2, 255, 259, 32, 64), (2, 300, 260, 32, 64), (2, 300, 260, 64, 32)])
def test_conv3x3_gradients(B, H, W, cin, cout):
    torch, ws, wo = _setup()
    rng = np.random.default_rng(7 + cin)
    x = rng.standard_normal((B, H, W, cin)).astype(np.float32)
    dy = rng.standard_normal((B, H, W, cout)).astype(np.float32)
    wt, wb, w4 = _weights(torch, ws, rng, cout, cin)
    xt, dyt = torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda()
    dw = torch.zeros((cout, 9 * cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    L = ws._lib()
    s = ws._stream(torch)
    assert L.asf_warm_conv3x3_wgrad(ws._ptr(xt), ws._ptr(dyt), ws._ptr(dw), ws._ptr(db), B, H, W, cin, cout, s) == 0
    # the float pixel-coordinate division is exact below 2^22 pixels; larger batches are refused
    assert L.asf_warm_conv3x3_wgrad(ws._ptr(xt), ws._ptr(dyt), ws._ptr(dw), ws._ptr(db), 1 << 22, 1, 1, cin, cout,
                                    s) == -1
    dw_o, db_o = wo.conv3x3_weight_grad(x, dy)
    e_w = _rel(dw.cpu().numpy().reshape(cout, 3, 3, cin), dw_o)
    e_b = _rel(db.cpu().numpy(), db_o)
    # input gradient: the forward with flipped, transposed weights
    flip = torch.empty_like(wb)
    assert L.asf_warm_flip_weights(ws._ptr(wb), ws._ptr(flip), cin, cout, s) == 0
    dx = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    if cin % 32 == 0:
        assert L.asf_warm_conv3x3(ws._ptr(dyt), ws._ptr(flip), None, ws._ptr(dx), B, H, W, cout, cin, 0, s) == 0
        e_x = _rel(dx.cpu().numpy(), wo.conv3x3_input_grad(dy, wo.bf16(w4)))
    else:
        e_x = 0.0
    print(f"grads {B}x{H}x{W} {cin}->{cout}: dw {e_w:.2e} db {e_b:.2e} dx {e_x:.2e}")
    assert e_w < 1e-5 and e_b < 1e-5 and e_x < 1e-5


# C = 5: the one-channel kernels; C = 8: four channels per thread (float4)
@pytest.mark.parametrize("C,src_off,dst_c,dst_off,count", [(5, 1, 9, 4, 3), (8, 4, 12, 8, 4)])
def test_pool_up_copy_relu_axpy(C, src_off, dst_c, dst_off, count):
    torch, ws, wo = _setup()
    rng = np.random.default_rng(3)
    L = ws._lib()
    s = ws._stream(torch)
    x = rng.standard_normal((2, 6, 10, C)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    p = torch.empty((2, 3, 5, C), dtype=torch.float32, device="cuda")
    assert L.asf_warm_pool2(ws._ptr(xt), ws._ptr(p), 2, 6, 10, C, s) == 0
    assert _rel(p.cpu().numpy(), wo.pool2(x)) < 1e-7
    pb = torch.empty_like(xt)
    assert L.asf_warm_pool2_backward(ws._ptr(p), ws._ptr(pb), 2, 6, 10, C, s) == 0
    assert _rel(pb.cpu().numpy(), wo.pool2_backward(p.cpu().numpy())) < 1e-7
    u = torch.empty((2, 12, 20, C), dtype=torch.float32, device="cuda")
    assert L.asf_warm_up2(ws._ptr(xt), ws._ptr(u), 2, 6, 10, C, s) == 0
    assert np.array_equal(u.cpu().numpy(), wo.up2(x))
    ub = torch.empty_like(xt)
    assert L.asf_warm_up2_backward(ws._ptr(u), ws._ptr(ub), 2, 6, 10, C, s) == 0
    assert _rel(ub.cpu().numpy(), wo.up2_backward(u.cpu().numpy())) < 1e-7
    dst = torch.zeros((2, 6, 10, dst_c), dtype=torch.float32, device="cuda")
    assert L.asf_warm_copy_channels(ws._ptr(xt), C, src_off, ws._ptr(dst), dst_c, dst_off, count, 120, s) == 0
    want = np.zeros((2, 6, 10, dst_c), dtype=np.float32)
    want[..., dst_off:dst_off + count] = x[..., src_off:src_off + count]
    assert np.array_equal(dst.cpu().numpy(), want)
    dy = torch.from_numpy(rng.standard_normal(x.shape).astype(np.float32)).cuda()
    dx = torch.empty_like(dy)
    assert L.asf_warm_relu_backward(ws._ptr(xt), ws._ptr(dy), ws._ptr(dx), x.size, s) == 0
    assert np.array_equal(dx.cpu().numpy(), np.where(x > 0, dy.cpu().numpy(), 0.0).astype(np.float32))
    y = dy.clone()
    assert L.asf_warm_axpy(ws._ptr(xt), ws._ptr(y), 0.5, x.size, s) == 0
    assert _rel(y.cpu().numpy(), dy.cpu().numpy() + 0.5 * x) < 1e-7


def test_adam_step():
    torch, ws, wo = _setup()
    rng = np.random.default_rng(4)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = rng.standard_normal(n).astype(np.float32) * 0.1
    v = np.abs(rng.standard_normal(n)).astype(np.float32) * 0.1
    pt, gt, mt, vt = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    pb = torch.empty(n, dtype=torch.int16, device="cuda")
    L = ws._lib()
    assert L.asf_warm_adam(ws._ptr(pt), ws._ptr(gt), ws._ptr(mt), ws._ptr(vt), ws._ptr(pb), n, 1e-2, 0.9, 0.999,
                           1e-8, 3, ws._stream(torch)) == 0
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    p2 = p - 1e-2 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    assert _rel(pt.cpu().numpy(), p2) < 1e-6
    assert np.array_equal(pb.cpu().numpy(), ws.bf16_bits(torch, pt).cpu().numpy())


def _oracle_params(net):
    params = []
    for i, (ci, co, _) in enumerate(net.shapes):
        wv = net.wb[i].cpu().numpy().astype(np.int32) & 0xFFFF
        w = (wv.astype(np.uint32) << 16).view(np.float32).astype(np.float64).reshape(co, 3, 3, ci)
        params.append((w, net.b[i].cpu().numpy().astype(np.float64)))
    return params


@pytest.mark.parametrize("side", [16, 256])
def test_infer_matches_forward(side):
    """Inference without kept activations (at 256^2 the three decoder concatenations are
    read in place by their convolutions, at 16^2 they are too small and concatenated):
    bit for bit the output of the training forward."""
    torch, ws, wo = _setup()
    net = ws.WarmNet(base=32, seed=4, head_scale=1.0)
    rng = np.random.default_rng(side)
    x = np.zeros((1, side, side, 16), dtype=np.float32)
    x[..., :2] = rng.standard_normal((1, side, side, 2))
    xt = torch.from_numpy(x).cuda()
    out, _ = net.forward(xt)
    assert np.array_equal(net.infer(xt).cpu().numpy(), out.cpu().numpy())


def test_network_forward_and_gradient():
    """The whole encoder-decoder on the GPU against the oracle network (same BF16
    weights, the same roundings).  Every layer is checked on the GPU's own data: its
    output from its input, its weight, bias and input gradients from its output
    gradient (the kernels' sums differ from the oracle's only in FP32 order).  The
    chain end to end is checked with a looser bar: the two sides' FP32 values
    differ in the last bits, which now and then rounds an activation to the other
    neighbouring BF16 value, and later layers carry those flips on."""
    torch, ws, wo = _setup()
    net = ws.WarmNet(base=32, seed=3, head_scale=1.0)
    rng = np.random.default_rng(5)
    B, H, W = 2, 16, 16
    x = np.zeros((B, H, W, 16), dtype=np.float32)
    x[..., :2] = rng.standard_normal((B, H, W, 2))
    out, cache = net.forward(torch.from_numpy(x).cuda())
    dout = rng.standard_normal(out.shape).astype(np.float32)
    net.zero_grad()
    rec = {}
    net.backward(torch.from_numpy(dout).cuda(), cache, record=rec)
    params = _oracle_params(net)
    worst = 0.0
    for i, (ci, co, relu) in enumerate(net.shapes):
        inp = cache["in"][i].cpu().numpy()
        ef = _rel(cache["a"][i].cpu().numpy(), wo.conv3x3(inp, params[i][0], params[i][1], relu=relu))
        dy, dpre, dx = (t.cpu().numpy() if t is not None else None for t in rec[i])
        assert np.array_equal(dpre, np.where(cache["a"][i].cpu().numpy() > 0, dy, 0.0)) if relu else True
        dw_o, db_o = wo.conv3x3_weight_grad(inp, dpre)
        ew = _rel(net.gw[i].cpu().numpy().reshape(co, 3, 3, ci), dw_o)
        eb = _rel(net.gb[i].cpu().numpy(), db_o)
        ex = _rel(dx, wo.conv3x3_input_grad(dpre, params[i][0])) if dx is not None else 0.0
        print(f"layer {i}: forward {ef:.1e} dw {ew:.1e} db {eb:.1e} dx {ex:.1e}")
        worst = max(worst, ef, ew, eb, ex)
    assert worst < 1e-5
    # end to end (wiring of pooling, upsampling, concatenation and skip gradients)
    o_ref, cache_ref = wo.net_forward(x, params)
    grads = wo.net_backward(dout, params, cache_ref)
    e_out = _rel(out.cpu().numpy(), o_ref)
    e_grad = max(_rel(net.gw[i].cpu().numpy().reshape(g[0].shape), g[0]) for i, g in enumerate(grads))
    print(f"end to end: output {e_out:.1e}, worst weight gradient {e_grad:.1e}")
    assert e_out < 1e-2 and e_grad < 1e-1


def test_trained_network_speeds_up_the_descent():
    """Train the network briefly through the forward and adjoint kernels on pairs the
    forward method generates (128^2 problems), then on held-out problems compare the
    adjoint descent from zero phase with the descent from the network's phase: the
    network's start has a lower loss, and its descent reaches the zero-phase descent's
    final loss in fewer iterations."""
    torch, ws, wo = _setup()
    pr = ws.HoloProblems(side=128, seed=0)
    rng = np.random.default_rng(1)
    pairs = [pr.make(rng)[:2] for _ in range(256)]
    net = ws.WarmNet(base=32, seed=0)
    losses = ws.train(net, pr, pairs, steps=300, lr=1e-3, batch=4, seed=2)
    print(f"training loss {np.mean(losses[:20]):.3f} -> {np.mean(losses[-20:]):.3f}")
    assert np.mean(losses[-20:]) < 0.8 * np.mean(losses[:20])
    erng = np.random.default_rng(99)
    iters = []
    for k in range(3):
        d, inten, _ = pr.make(erng)
        lz, lw = ws.compare_descent(net, pr, d, inten, steps=50, lr=0.05)
        it = ws.iterations_to_reach(lw, lz[-1])
        iters.append(it)
        print(f"held-out {k}: zero {lz[0]:.3f} -> {lz[-1]:.4f}, warm {lw[0]:.3f} -> {lw[-1]:.4f}, "
              f"warm reaches the zero-phase final loss at iteration {it}")
        assert lw[0] < lz[0]
    # every held-out problem: the warm descent reaches the zero-phase descent's final
    # loss (same target, same scale) before the last of its 50 iterations
    assert all(it is not None and it < 50 for it in iters), iters
    assert np.mean(iters) < 40
