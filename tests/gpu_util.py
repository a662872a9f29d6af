"""Helpers shared by the GPU tests (no method arithmetic: inputs and norms)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)
