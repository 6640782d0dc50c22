"""CPU pins of the warm-start network oracle (oracle/warm_oracle.py): a brute-force
convolution, finite differences of the whole network's backward, adjoint
identities of pooling and upsampling, and BF16 rounding on known values."""
import numpy as np

from oracle import warm_oracle as wo


def test_bf16_rounding_known_values():
    # BF16 keeps 7 fraction bits: neighbours of 1 are 1 - 2^-8, 1 and 1 + 2^-7
    x = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5,
                  1.0 + 2 ** -8 + 2 ** -20], dtype=np.float32)
    # exact; tie to even (down); tie to even (up to 1 + 2^-6); below half; exact; above a tie
    want = np.array([1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 1.0 + 2 ** -7])
    assert np.array_equal(wo.bf16(x), want)


def test_conv_against_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 4, 3))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    ref = np.zeros((2, 5, 4, 2))
    for n in range(2):
        for y in range(5):
            for xx in range(4):
                for o in range(2):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            yy, xq = y + ky - 1, xx + kx - 1
                            if 0 <= yy < 5 and 0 <= xq < 4:
                                s += np.dot(x[n, yy, xq], w[o, ky, kx])
                    ref[n, y, xx, o] = s
    assert np.abs(wo.conv3x3(x, w, b, rounded=False) - ref).max() < 1e-12
    assert np.abs(wo.conv3x3(x, w, b, relu=True, rounded=False) - np.maximum(ref, 0.0)).max() < 1e-12


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(wo.pool2(x) * y) - np.sum(x * wo.pool2_backward(y))) < 1e-12
    z = rng.standard_normal((2, 12, 16, 3))
    assert abs(np.sum(wo.up2(x) * z) - np.sum(x * wo.up2_backward(z))) < 1e-12


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 5, 6, 4))
    w = rng.standard_normal((3, 3, 3, 4))
    dy = rng.standard_normal((1, 5, 6, 3))
    # <conv(x), dy> = <x, input_grad(dy)> and = <w, weight_grad(x, dy)>
    lhs = np.sum(wo.conv3x3(x, w, rounded=False) * dy)
    assert abs(lhs - np.sum(x * wo.conv3x3_input_grad(dy, w, rounded=False))) < 1e-10
    assert abs(lhs - np.sum(w * wo.conv3x3_weight_grad(x, dy, rounded=False)[0])) < 1e-10


def test_network_backward_against_finite_differences():
    rng = np.random.default_rng(3)
    shapes = wo.layer_shapes(c=4, cin0=2, cout_head=2)
    params = [(rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci)), rng.standard_normal(co) * 0.1 + 0.05)
              for ci, co, _ in shapes]
    x = rng.standard_normal((1, 8, 8, 2))
    out, cache = wo.net_forward(x, params, rounded=False)
    dout = rng.standard_normal(out.shape)
    grads = wo.net_backward(dout, params, cache, rounded=False)
    checked = 0
    for li in range(len(shapes)):
        w, b = params[li]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            e = 1e-6
            vals = []
            for sgn in (1, -1):
                wp = w.copy()
                wp[idx] += sgn * e
                P = list(params)
                P[li] = (wp, b)
                vals.append(np.sum(dout * wo.net_forward(x, P, rounded=False)[0]))
            fd = (vals[0] - vals[1]) / (2 * e)
            an = grads[li][0][idx]
            assert abs(fd - an) <= 1e-6 * (1 + abs(an)), (li, idx, fd, an)
            checked += 1
        # bias
        j = int(rng.integers(0, b.shape[0]))
        vals = []
        for sgn in (1, -1):
            bp = b.copy()
            bp[j] += sgn * 1e-6
            P = list(params)
            P[li] = (w, bp)
            vals.append(np.sum(dout * wo.net_forward(x, P, rounded=False)[0]))
        assert abs((vals[0] - vals[1]) / 2e-6 - grads[li][1][j]) <= 1e-6 * (1 + abs(grads[li][1][j]))
    assert checked == 3 * len(shapes)
