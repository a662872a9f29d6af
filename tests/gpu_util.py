"""Helpers shared by the GPU tests (no method arithmetic: inputs and norms)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b):
    """max_k |a_k - b_k| / max_k |b_k|: the worst single element, on the scale
    of the largest reference value."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def assert_close(got, want, tol, what=""):
    """Element-wise parity: both the norm-wise relative error and the worst
    element (relative to the largest reference magnitude) are within tol."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    en, em = rel(got, want), max_rel(got, want)
    if what:
        say(f"  {what}: rel {en:.2e}  max {em:.2e}  (tol {tol:.0e})")
    assert en <= tol, f"{what}: norm-wise {en:.3e} > {tol:.1e}"
    assert em <= tol, f"{what}: element-wise {em:.3e} > {tol:.1e}"


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)
