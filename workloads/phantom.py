"""Random-ellipse phantoms on [-1/2, 1/2]^2 and their cell averages."""
from __future__ import annotations

import numpy as np


def ellipse_phantom_params(seed: int, n_ellipses: int = 10):
    rng = np.random.default_rng(seed)
    return {
        "centre": rng.uniform(-0.35, 0.35, size=(n_ellipses, 2)),
        "axes": rng.uniform(0.03, 0.3, size=(n_ellipses, 2)),
        "angle": rng.uniform(0, np.pi, size=n_ellipses),
        "amp": rng.uniform(-1, 1, size=n_ellipses),
        "wave": rng.uniform(-3, 3, size=2),
    }


def phantom_eval(params, x, y):
    """f(x, y) = (sum of ellipse indicators * amplitudes) * (1 + 0.2 sin(2 pi a.x))."""
    f = np.zeros(np.broadcast(x, y).shape)
    for c, ax, an, am in zip(params["centre"], params["axes"], params["angle"], params["amp"]):
        dx, dy = x - c[0], y - c[1]
        ca, sa = np.cos(an), np.sin(an)
        u = (ca * dx + sa * dy) / ax[0]
        v = (-sa * dx + ca * dy) / ax[1]
        f = f + am * ((u * u + v * v) <= 1.0)
    a = params["wave"]
    return f * (1 + 0.2 * np.sin(2 * np.pi * (a[0] * x + a[1] * y)))


def phantom_cell_averages(params, J: int, sub: int = 4) -> np.ndarray:
    """x0[i, j] = 2^-J * mean of f over a sub x sub sample of dyadic cell (i, j),
    cell i covering [(i - N/2)/N, (i - N/2 + 1)/N) along x (row index i = x)."""
    N = 1 << J
    off = (np.arange(sub) + 0.5) / sub
    c = (np.arange(N)[:, None] - N / 2 + off[None, :]) / N          # (N, sub)
    xs = c.reshape(-1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    f = phantom_eval(params, X, Y).reshape(N, sub, N, sub).mean(axis=(1, 3))
    return (2.0 ** (-J)) * f


def phantom_cell_averages_torch(params_list, J: int, device, sub: int = 4):
    """The same cell averages as ``phantom_cell_averages`` for a list of
    phantoms at once, evaluated with torch on ``device`` (FP64).  Returns a
    (len(params_list), N, N) float64 tensor.  Input generation only: used to
    make thousands of training phantoms quickly."""
    import torch
    N = 1 << J
    off = (torch.arange(sub, dtype=torch.float64, device=device) + 0.5) / sub
    c = ((torch.arange(N, dtype=torch.float64, device=device)[:, None] - N / 2 + off[None, :]) / N).reshape(-1)
    X, Y = torch.meshgrid(c, c, indexing="ij")
    out = torch.empty((len(params_list), N, N), dtype=torch.float64, device=device)
    for k, prm in enumerate(params_list):
        f = torch.zeros_like(X)
        for ce, ax, an, am in zip(prm["centre"], prm["axes"], prm["angle"], prm["amp"]):
            dx, dy = X - float(ce[0]), Y - float(ce[1])
            ca, sa = float(np.cos(an)), float(np.sin(an))
            u = (ca * dx + sa * dy) / float(ax[0])
            v = (-sa * dx + ca * dy) / float(ax[1])
            f = f + float(am) * ((u * u + v * v) <= 1.0).to(torch.float64)
        a = prm["wave"]
        f = f * (1 + 0.2 * torch.sin(2 * np.pi * (float(a[0]) * X + float(a[1]) * Y)))
        out[k] = (2.0 ** (-J)) * f.reshape(N, sub, N, sub).mean(dim=(1, 3))
    return out
