"""GPU warm-start network (gs_cnn_*) against the CNN oracle.

The oracle is run twice: with bf16 rounding at the GPU's storage points
(emulate=True), which isolates the kernels' FP32 accumulation order, and in
plain FP64.  Tolerances (norm-wise relative):
  * network correction (output minus input): <= 2e-3 against the emulating
    oracle (a stored bf16 value can land one unit in the 8th bit apart when
    an FP32 sum sits near a rounding boundary), <= 3e-2 against FP64 (bf16
    storage of 5 activation layers: 5 roundings of relative size <= 2^-9);
  * weight gradients per layer: <= 5e-3 emulating; <= 1e-1 against FP64, a
    sanity bound only: the gradient of layer 1 passes through up to ten bf16
    roundings (five activations, five deltas, 2^-9 relative each), and on
    a handful of pixels these do not average out;
  * Adam step: <= 1e-5 of the weights (FP32 against FP64 arithmetic).
Shapes cover one tile, ragged tiles (sides not multiples of 16), a single
row, several images, the full 256 x 256 images of the warm-start workload,
and 40 ragged 80 x 72 images: 1000 tiles, more than the convolution and
weight-gradient kernels have workgroups (two per CU), so workgroups walk
several tiles across image borders with the next tile's loads in flight, and
2560 row segments for the thin-layer gradient's 1024 workgroups."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cnn as ocnn

from gpu_util import crandn, rel, to_dev, to_host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs as _gs
    return _gs


def _weights(seed, last_scale=0.5):
    rng = np.random.default_rng(seed)
    parts = []
    for s in ocnn.layer_shapes():
        std = np.sqrt(2.0 / (9 * s[2]))
        parts.append(rng.standard_normal(s) * std)
    parts[-1] *= last_scale
    return ocnn.flatten(parts).astype(np.float32)


def _c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


SHAPES = [(1, 16, 16), (2, 20, 37), (3, 33, 17), (1, 1, 5), (2, 256, 256), (40, 80, 72)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(gs, shape):
    B, H, W = shape
    say(f"[cnn fwd] {shape}")
    rng = np.random.default_rng(100 + H + W)
    w = _weights(1 + B)
    u = _c64(crandn(rng, (B, H, W)))
    net = gs.Cnn(H, W, B)
    net.set_weights(w)
    out = to_host(net.forward(to_dev(u, torch.complex64)))
    ws = ocnn.unflatten(w.astype(np.float64))
    want_e = ocnn.to_complex(ocnn.forward(ws, u, emulate=True)[0])
    want_x = ocnn.to_complex(ocnn.forward(ws, u, emulate=False)[0])
    assert rel(out - u, want_e - u) < 2e-3
    assert rel(out - u, want_x - u) < 3e-2
    # complex128 in and out: the same network value up to the input rounding
    out64 = to_host(net.forward(to_dev(u, torch.complex128), out_dtype=torch.complex128))
    assert out64.dtype == np.complex128
    assert rel(out64 - u, want_e - u) < 2e-3
    net.destroy()


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_matches_oracle(gs, shape):
    B, H, W = shape
    say(f"[cnn bwd] {shape}")
    rng = np.random.default_rng(200 + H + W)
    w = _weights(2 + B)
    u = _c64(crandn(rng, (B, H, W)))
    t = _c64(u + 0.3 * crandn(rng, (B, H, W)))
    net = gs.Cnn(H, W, B)
    net.set_weights(w)
    net.forward(to_dev(u, torch.complex64), train=True)
    loss = net.backward(to_dev(t, torch.complex64))
    g = net.get_grads().astype(np.float64)
    ws = ocnn.unflatten(w.astype(np.float64))
    out_e, cache_e = ocnn.forward(ws, u, emulate=True)
    out_x, cache_x = ocnn.forward(ws, u, emulate=False)
    assert abs(loss - ocnn.loss(out_e, t)) <= 1e-3 * ocnn.loss(out_e, t)
    ge = ocnn.backward(cache_e, out_e, t, emulate=True)
    gx = ocnn.backward(cache_x, out_x, t, emulate=False)
    gg = ocnn.unflatten(g)
    errs = [(rel(gg[l], ge[l]), rel(gg[l], gx[l])) for l in range(ocnn.N_LAYERS)]
    for l, (e, x) in enumerate(errs):
        say(f"  layer {l + 1}: emulated {e:.2e}  fp64 {x:.2e}")
    for l, (e, x) in enumerate(errs):
        assert e < 5e-3, l
        assert x < 1e-1, l
    net.destroy()


def test_adam_step_matches_oracle(gs):
    say("[cnn adam]")
    B, H, W = 2, 24, 40
    rng = np.random.default_rng(300)
    w = _weights(3)
    u = _c64(crandn(rng, (B, H, W)))
    t = _c64(u + 0.3 * crandn(rng, (B, H, W)))
    net = gs.Cnn(H, W, B)
    net.set_weights(w)
    ws = ocnn.unflatten(w.astype(np.float64))
    m = [np.zeros_like(a) for a in ws]
    v = [np.zeros_like(a) for a in ws]
    for k in (1, 2, 3):
        net.forward(to_dev(u, torch.complex64), train=True)
        net.backward(to_dev(t, torch.complex64), want_loss=False)
        g = ocnn.unflatten(net.get_grads().astype(np.float64))
        net.step(1e-3)
        ws, m, v = ocnn.adam_step(ws, g, m, v, k, 1e-3)
        got = net.get_weights().astype(np.float64)
        want = ocnn.flatten(ws)
        assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want)), k
        # continue from the GPU's weights so the next gradients agree
        ws = ocnn.unflatten(got)
    gm, gv, st = net.get_state()
    assert st == 3
    assert rel(gm, ocnn.flatten(m)) < 1e-5 and rel(gv, ocnn.flatten(v)) < 1e-4
    net.destroy()


def test_deterministic_and_state_errors(gs):
    say("[cnn determinism]")
    B, H, W = 2, 40, 24
    rng = np.random.default_rng(400)
    net = gs.Cnn(H, W, B)
    net.set_weights(_weights(4))
    u = to_dev(crandn(rng, (B, H, W)), torch.complex64)
    t = to_dev(crandn(rng, (B, H, W)), torch.complex64)
    res = []
    for _ in range(2):
        o = to_host(net.forward(u, train=True, out_dtype=torch.complex64))
        net.backward(t, want_loss=False)
        res.append((o, net.get_grads()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    # backward needs a training forward of the same batch; batch is bounded
    net.forward(u)
    with pytest.raises(gs.GSError):
        net.backward(t)
    x3 = to_dev(crandn(rng, (3, H, W)), torch.complex64)
    with pytest.raises(ValueError):            # the binding refuses a batch above max_batch
        net.forward(x3)
    import ctypes
    o3 = torch.empty_like(x3)                  # and so does the library itself
    rc = gs.library().gs_cnn_forward(net.handle, ctypes.c_void_p(x3.data_ptr()), ctypes.c_void_p(o3.data_ptr()),
                                     3, 0, None)
    assert rc == gs.GS_ERR_INVALID_ARG
    net.destroy()


def test_training_reduces_loss(gs):
    """The training loop itself: 150 Adam steps on a fixed batch whose target
    is a fixed local linear map of the input (a 3 x 3 box average)."""
    say("[cnn train]")
    B, H, W = 8, 32, 32
    rng = np.random.default_rng(500)
    u = crandn(rng, (B, H, W))
    pad = np.pad(u, ((0, 0), (1, 1), (1, 1)))
    t = sum(pad[:, dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)) / 9.0
    net = gs.Cnn(H, W, B)
    net.set_weights(_weights(5, last_scale=0.1))
    ud, td = to_dev(u, torch.complex64), to_dev(t, torch.complex64)
    losses = []
    for k in range(150):
        net.forward(ud, train=True)
        losses.append(net.backward(td))
        net.step(2e-3)
    say(f"  loss {losses[0]:.3f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
    net.destroy()


def test_backward_complex128_target(gs):
    """Targets given as complex128 (GS_CNN_TGT_F64) against the emulating oracle."""
    say("[cnn bwd f64 target]")
    B, H, W = 2, 18, 21
    rng = np.random.default_rng(600)
    w = _weights(6)
    u = _c64(crandn(rng, (B, H, W)))
    t = u + 0.3 * crandn(rng, (B, H, W))            # complex128, not rounded to FP32
    net = gs.Cnn(H, W, B)
    net.set_weights(w)
    net.forward(to_dev(u, torch.complex64), train=True)
    loss = net.backward(to_dev(t, torch.complex128))
    ws = ocnn.unflatten(w.astype(np.float64))
    out_e, cache_e = ocnn.forward(ws, u, emulate=True)
    assert abs(loss - ocnn.loss(out_e, t)) <= 1e-3 * ocnn.loss(out_e, t)
    ge = ocnn.backward(cache_e, out_e, t, emulate=True)
    gg = ocnn.unflatten(net.get_grads().astype(np.float64))
    for l in range(ocnn.N_LAYERS):
        assert rel(gg[l], ge[l]) < 5e-3, l
    net.destroy()


def test_checkpoint_resume_is_exact(gs, tmp_path):
    """Weights and Adam state saved after 3 steps and loaded into a new
    handle continue training bit for bit like the original handle."""
    say("[cnn checkpoint]")
    B, H, W = 2, 24, 24
    rng = np.random.default_rng(700)
    u = to_dev(crandn(rng, (B, H, W)), torch.complex64)
    t = to_dev(crandn(rng, (B, H, W)), torch.complex64)
    a = gs.Cnn(H, W, B)
    a.set_weights(_weights(7))
    a.input_scale = 0.75
    for _ in range(3):
        a.forward(u, train=True)
        a.backward(t, want_loss=False)
        a.step(1e-3)
    path = str(tmp_path / "ckpt.npz")
    a.save(path)
    b = gs.Cnn(H, W, B)
    b.load(path)
    assert b.input_scale == a.input_scale
    for net in (a, b):
        for _ in range(2):
            net.forward(u, train=True)
            net.backward(t, want_loss=False)
            net.step(1e-3)
    assert np.array_equal(a.get_weights(), b.get_weights())
    ma, va, sa = a.get_state()
    mb, vb, sb = b.get_state()
    assert sa == sb == 5 and np.array_equal(ma, mb) and np.array_equal(va, vb)
    a.destroy()
    b.destroy()
