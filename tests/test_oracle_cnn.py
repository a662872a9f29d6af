"""Pins of the CNN oracle (oracle/cnn.py) against definitions outside it:
brute-force loops, a library correlation, adjoint identities, finite
differences, the closed form of Adam under a constant gradient, and the
rounding rule of bfloat16."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_bf16_round_definition():
    # 8 significant bits; ties go to the even neighbour
    one = 1.0
    assert cnn.bf16_round(one) == one
    assert cnn.bf16_round(1 + 2.0 ** -8) == 1.0                      # tie -> even (1.0)
    assert cnn.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6        # tie -> even (1 + 2^-6)
    assert cnn.bf16_round(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert cnn.bf16_round(-1 - 2.0 ** -7) == -1 - 2.0 ** -7           # representable
    assert cnn.bf16_round(3.0 * 2.0 ** -130) == 3.0 * 2.0 ** -130     # subnormal range, 2 bits
    r = np.random.default_rng(1).standard_normal(10000) * 1e3
    q = cnn.bf16_round(r)
    # |q - r| <= half a unit in the 8th bit
    e = np.floor(np.log2(np.abs(r)))
    assert np.all(np.abs(q - r) <= 2.0 ** (e - 8) * (1 + 1e-12))


def _brute_conv(a, w):
    B, H, W, Ci = a.shape
    Co = w.shape[3]
    z = np.zeros((B, H, W, Co))
    for b in range(B):
        for y in range(H):
            for x in range(W):
                for co in range(Co):
                    s = 0.0
                    for ky in range(3):
                        for kx in range(3):
                            yy, xx = y + ky - 1, x + kx - 1
                            if 0 <= yy < H and 0 <= xx < W:
                                for ci in range(Ci):
                                    s += a[b, yy, xx, ci] * w[ky, kx, ci, co]
                    z[b, y, x, co] = s
    return z


def test_conv_matches_brute_force():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((2, 3, 5, 2))
    w = rng.standard_normal((3, 3, 2, 3))
    assert np.allclose(cnn.conv3x3(a, w), _brute_conv(a, w), rtol=1e-13, atol=1e-13)


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((1, 7, 6, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    want = np.zeros((7, 6, 4))
    for co in range(4):
        for ci in range(3):
            want[:, :, co] += correlate2d(a[0, :, :, ci], w[:, :, ci, co], mode="same", boundary="fill")
    assert np.allclose(cnn.conv3x3(a, w)[0], want, rtol=1e-13, atol=1e-12)


def test_adjoint_identities():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 6, 5, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    d = rng.standard_normal((2, 6, 5, 4))
    lhs = np.sum(cnn.conv3x3(a, w) * d)
    assert abs(lhs - np.sum(a * cnn.conv3x3_adjoint(d, w))) < 1e-11 * abs(lhs)
    assert abs(lhs - np.sum(w * cnn.conv3x3_weight_grad(a, d))) < 1e-11 * abs(lhs)


def _init(hidden, rng, last_scale=1.0):
    ws = []
    for k, s in enumerate(cnn.layer_shapes(hidden)):
        std = np.sqrt(2.0 / (9 * s[2]))
        ws.append(rng.standard_normal(s) * std * (last_scale if k == cnn.N_LAYERS - 1 else 1.0))
    return ws


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    hidden = 4
    ws = _init(hidden, rng)
    u = rng.standard_normal((2, 6, 7)) + 1j * rng.standard_normal((2, 6, 7))
    t = rng.standard_normal((2, 6, 7)) + 1j * rng.standard_normal((2, 6, 7))

    def L(wlist):
        out, _ = cnn.forward(wlist, u, emulate=False)
        return cnn.loss(out, t)

    out, cache = cnn.forward(ws, u, emulate=False)
    g = cnn.backward(cache, out, t, emulate=False)
    h = 1e-6
    for l in range(cnn.N_LAYERS):
        for _ in range(4):
            idx = tuple(rng.integers(0, n) for n in ws[l].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h
            wm[l][idx] -= h
            fd = (L(wp) - L(wm)) / (2 * h)
            assert abs(fd - g[l][idx]) <= 1e-6 * max(1e-3, abs(fd)), (l, idx, fd, g[l][idx])


def test_residual_form_and_homogeneity():
    rng = np.random.default_rng(6)
    ws = _init(8, rng)
    u = rng.standard_normal((1, 5, 5)) + 1j * rng.standard_normal((1, 5, 5))
    zero_last = [w.copy() for w in ws]
    zero_last[-1][:] = 0
    out, _ = cnn.forward(zero_last, u, emulate=False)
    assert np.array_equal(cnn.to_complex(out), u)
    o1, _ = cnn.forward(ws, u, emulate=False)
    o2, _ = cnn.forward(ws, 3.5 * u, emulate=False)
    assert np.allclose(o2, 3.5 * o1, rtol=1e-13, atol=1e-13)


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g, m_hat = g and v_hat = g^2 at every step, so
    each step moves w by exactly lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    w0 = [rng.standard_normal((3, 3, 2, 2))]
    g = [rng.standard_normal((3, 3, 2, 2))]
    w, m, v = w0, [np.zeros_like(w0[0])], [np.zeros_like(w0[0])]
    lr, eps = 1e-3, 1e-8
    for k in range(1, 6):
        w, m, v = cnn.adam_step(w, g, m, v, k, lr, eps=eps)
    want = w0[0] - 5 * lr * g[0] / (np.abs(g[0]) + eps)
    assert np.allclose(w[0], want, rtol=1e-12, atol=1e-15)


def test_flatten_roundtrip_and_sizes():
    shapes = cnn.layer_shapes()
    assert [int(np.prod(s)) for s in shapes] == [576, 9216, 9216, 9216, 9216, 576]
    rng = np.random.default_rng(8)
    ws = _init(32, rng)
    flat = cnn.flatten(ws)
    assert flat.size == 38016
    back = cnn.unflatten(flat)
    assert all(np.array_equal(a, b) for a, b in zip(ws, back))
