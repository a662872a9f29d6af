"""FP64 reference of the learned warm start: a small residual CNN that maps
the adjoint image A^H b = T^H W y of a generalized-sampling problem to an
estimate of its least-squares solution, used as the CGLS start x0.

TEST INFRASTRUCTURE ONLY (see the package header).  This is not from the
paper: the paper solves from x0 = 0.  The network, its training loss and its
optimizer are this build's choices, restated here from their standard
definitions so that the GPU kernels have something independent to match:

* 3 x 3 convolution (cross-correlation), stride 1, zero padding 1,
  channels-last (B, H, W, C), weights w[ky, kx, ci, co]:
      z[b, y, x, co] = sum_{dy, dx in {-1,0,1}} sum_ci
                       a[b, y+dy, x+dx, ci] * w[dy+1, dx+1, ci, co],
  a taken as 0 outside the image.  No biases (the map from A^H b to the LS
  solution is linear, and a bias-free ReLU net is positively homogeneous).
* Network: the complex image u becomes two real channels (re, im),
  multiplied by a fixed scale s; conv 2->C, ReLU; four times conv C->C,
  ReLU; conv C->2; output = s u + last conv (residual form).  C = 32.
* Loss: relative squared error over the batch,
      L = sum_b ||out_b - t_b||^2 / sum_b ||t_b||^2.
* Backward by the chain rule, written out per layer (no autodiff).
* Adam (Kingma and Ba, 2015, Algorithm 1) with bias correction.

Storage precision.  The GPU stores hidden activations and hidden-layer
gradients in bfloat16 (round to nearest even from FP32), multiplies with
bf16 copies of the FP32 master weights, and accumulates in FP32.  With
``emulate=True`` the oracle rounds at exactly those storage points (values
carried in FP64 otherwise), so a comparison isolates the kernels' own
arithmetic; with ``emulate=False`` everything is FP64.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 32
N_LAYERS = 6


def bf16_round(a):
    """Round to the nearest bfloat16 (8 significant bits, ties to even), via
    FP32 as the GPU does (FP32 result -> bf16).  Finite inputs only."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def layer_shapes(hidden: int = HIDDEN):
    ch = [2] + [hidden] * (N_LAYERS - 1) + [2]
    return [(3, 3, ch[i], ch[i + 1]) for i in range(N_LAYERS)]


def _shift(a, dy, dx):
    """s[b, y, x, c] = a[b, y+dy, x+dx, c], zero outside the image."""
    B, H, W, C = a.shape
    s = np.zeros_like(a)
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    s[:, yd, xd, :] = a[:, ys, xs, :]
    return s


def conv3x3(a, w):
    """z = sum over the 9 taps of shift(a, dy, dx) @ w[dy+1, dx+1]."""
    z = np.zeros(a.shape[:3] + (w.shape[3],))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            z += _shift(a, dy, dx) @ w[dy + 1, dx + 1]
    return z


def conv3x3_adjoint(d, w):
    """Adjoint of conv3x3 in its input: g[q, ci] = sum_t sum_co d[q - t, co] w[t, ci, co]."""
    g = np.zeros(d.shape[:3] + (w.shape[2],))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            g += _shift(d, -dy, -dx) @ w[dy + 1, dx + 1].T
    return g


def conv3x3_weight_grad(a, d):
    """Adjoint of conv3x3 in its weights: dw[t, ci, co] = sum_{b,p} a[p + t, ci] d[p, co]."""
    dw = np.zeros((3, 3, a.shape[3], d.shape[3]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            s = _shift(a, dy, dx)
            dw[dy + 1, dx + 1] = s.reshape(-1, a.shape[3]).T @ d.reshape(-1, d.shape[3])
    return dw


def to_channels(u):
    """(B, H, W) complex -> (B, H, W, 2) real (re, im)."""
    u = np.asarray(u)
    return np.stack([u.real, u.imag], axis=-1).astype(np.float64)


def to_complex(a):
    return a[..., 0] + 1j * a[..., 1]


def forward(weights, u, emulate: bool = True, scale: float = 1.0):
    """Returns (out as (B, H, W, 2), cache).  u: (B, H, W) complex; the
    network sees scale * u (FP32: the input rounded to FP32, then scaled)."""
    rnd = bf16_round if emulate else (lambda v: v)
    a = f32(f32(to_channels(u)) * f32(scale)) if emulate else scale * to_channels(u)
    acts = [a]
    wq = [rnd(w) for w in weights]
    for l in range(N_LAYERS - 1):
        a = rnd(np.maximum(conv3x3(a, wq[l]), 0.0))
        acts.append(a)
    z = conv3x3(a, wq[-1])
    out = acts[0] + z
    if emulate:
        out = f32(out)
    return out, {"acts": acts, "wq": wq}


def loss(out, target):
    t = to_channels(target) if np.iscomplexobj(target) else np.asarray(target, float)
    return float(np.sum((out - t) ** 2) / np.sum(t * t))


def backward(cache, out, target, emulate: bool = True):
    """Gradients of ``loss`` with respect to the six weight tensors (the
    master weights: the bf16 copies have the same gradient)."""
    rnd = bf16_round if emulate else (lambda v: v)
    t = to_channels(target) if np.iscomplexobj(target) else np.asarray(target, float)
    acts, wq = cache["acts"], cache["wq"]
    S = np.sum(t * t)
    d = 2.0 * (out - t) / S
    if emulate:
        d = f32(d)
    grads = [None] * N_LAYERS
    for l in range(N_LAYERS - 1, -1, -1):
        grads[l] = conv3x3_weight_grad(acts[l], d)
        if l == 0:
            break
        g = conv3x3_adjoint(d, wq[l])
        d = rnd(g * (acts[l] > 0))
    return grads


def adam_step(weights, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (weights, m, v)."""
    nw, nm, nv = [], [], []
    for w, g, mi, vi in zip(weights, grads, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mhat = mi / (1 - beta1 ** step)
        vhat = vi / (1 - beta2 ** step)
        nw.append(w - lr * mhat / (np.sqrt(vhat) + eps))
        nm.append(mi)
        nv.append(vi)
    return nw, nm, nv


def flatten(weights):
    return np.concatenate([np.asarray(w, float).reshape(-1) for w in weights])


def unflatten(flat, hidden: int = HIDDEN):
    out, k = [], 0
    for s in layer_shapes(hidden):
        n = int(np.prod(s))
        out.append(np.asarray(flat[k:k + n], float).reshape(s))
        k += n
    return out
