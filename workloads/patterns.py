"""Sampling patterns in the frequency domain (unnormalized frequencies xi)."""
from __future__ import annotations

import math

import numpy as np


def grid(M: int, eps: float) -> np.ndarray:
    """Uniform points eps * (-M/2 .. M/2 - 1) (the paper's ``grid(M, eps)``)."""
    return eps * (np.arange(M, dtype=np.float64) - M // 2)


def jitter_1d(M: int, spacing: float, seed: int) -> np.ndarray:
    """xi_k = (k + u_k) * spacing, k = -M/2 .. M/2-1, u_k ~ U(-1/4, 1/4)."""
    rng = np.random.default_rng(seed)
    k = np.arange(M, dtype=np.float64) - M // 2
    return (k + rng.uniform(-0.25, 0.25, size=M)) * spacing


def _arc_length(theta, a):
    return 0.5 * a * (theta * np.sqrt(1 + theta * theta) + np.arcsinh(theta))


def spiral_2d(interleaves: int, per_arm: int, r_max: float, arm_gap: float = 0.5) -> np.ndarray:
    """Interleaved Archimedean spiral r = a theta, a = interleaves*arm_gap/(2 pi),
    so neighbouring arms are arm_gap apart; points equally spaced in arc length
    at s = (t + 1/2) S / per_arm (the half offset keeps the arms from sharing a
    point at the origin); arm l is rotated by 2 pi l / interleaves.
    Returns (interleaves*per_arm, 2), arm-major order."""
    a = interleaves * arm_gap / (2 * math.pi)
    th_max = r_max / a
    S = _arc_length(th_max, a)
    s = (np.arange(per_arm) + 0.5) * S / per_arm
    th = np.sqrt(2 * s / a)                       # initial guess (s ~ a th^2 / 2)
    for _ in range(60):
        f = _arc_length(th, a) - s
        fp = a * np.sqrt(1 + th * th)
        th = th - f / fp
    r = a * th
    out = np.empty((interleaves * per_arm, 2))
    for l in range(interleaves):
        ang = th + 2 * math.pi * l / interleaves
        out[l * per_arm:(l + 1) * per_arm, 0] = r * np.cos(ang)
        out[l * per_arm:(l + 1) * per_arm, 1] = r * np.sin(ang)
    return out


def jitter_2d(M: int, half_width: float, seed: int) -> np.ndarray:
    """s x s grid (s = round(sqrt(M))) on [-half_width, half_width)^2 with
    spacing h = 2 half_width / s, each coordinate jittered by U(-1/4, 1/4) h."""
    rng = np.random.default_rng(seed)
    s = int(round(math.sqrt(M)))
    h = 2.0 * half_width / s
    c = (np.arange(s) - s / 2 + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    pts += rng.uniform(-0.25, 0.25, size=pts.shape) * h
    return pts
