"""The five workload configurations (inputs only; the data y = T x0 is formed
by whichever side consumes the inputs).

C1  1D db2, J=8, 1024 uniform points xi = k/2, unit weights, x0 ~ N(0,1),
    y = T x0 + complex N(0, (1e-8)^2) noise; CGLS tol 1e-10.
C2  1D db4, J=14, 65536 jittered points xi = (k + U(-1/4,1/4))/2,
    Voronoi lengths clipped to [-16384.25, 16384.25],
    x0_i ~ N(0,1) / (1 + |i - 8192|/512), noiseless y; tol 1e-8.
C3  2D db4, J=9, 1,048,576 spiral points (64 arms x 16384, r_max 256),
    Voronoi areas in the disk of radius 256.25, ellipse phantom x0,
    y = T x0 (complex64) + 1e-4 relative noise; tol 1e-6.
C4  one of 64 batched 2D problems: p in {2,4}, J in 6..9, jitter or spiral,
    M = round(U(2,4) 4^J), Voronoi weights, ellipse phantom; tol 1e-6.
C5  2D db4, J=8, 262,144 spiral points (64 arms x 4096, r_max 128).
"""
from __future__ import annotations

import math

import numpy as np

from .patterns import grid, jitter_1d, spiral_2d, jitter_2d
from .weights import voronoi_weights_1d, voronoi_weights_2d
from .phantom import ellipse_phantom_params, phantom_cell_averages


def complex_noise(n: int, sigma: float, seed: int) -> np.ndarray:
    """i.i.d. N(0, sigma^2) on the real and the imaginary parts."""
    rng = np.random.default_rng(seed)
    return sigma * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


def relative_noise(y: np.ndarray, rel: float, seed: int) -> np.ndarray:
    """n = rel * ||y|| / sqrt(2M) * (g1 + i g2), so ||n|| ~ rel ||y||."""
    M = y.size
    return complex_noise(M, rel * float(np.linalg.norm(y)) / math.sqrt(2 * M), seed)


def config_c1(J: int = 8, M: int = 1024):
    rng = np.random.default_rng(101)
    return {
        "name": "c1", "dim": 1, "J": J, "p": 2,
        "xi": grid(M, 0.5), "mu": None,
        "x0": rng.standard_normal(1 << J).astype(np.complex128),
        "noise_sigma": 1e-8, "noise_seed": 102, "tol": 1e-10,
    }


def config_c2(J: int = 14, M: int = 65536):
    N = 1 << J
    xi = jitter_1d(M, 0.5, 201)
    rng = np.random.default_rng(202)
    i = np.arange(N)
    x0 = rng.standard_normal(N) / (1 + np.abs(i - N / 2) / 512)
    K = M * 0.25 + 0.25
    return {
        "name": "c2", "dim": 1, "J": J, "p": 4,
        "xi": xi, "mu": voronoi_weights_1d(xi, K),
        "x0": x0.astype(np.complex128), "noise_sigma": 0.0, "tol": 1e-8,
    }


def spiral_problem(J: int, p: int, arms: int, per_arm: int, r_max: float, phantom_seed: int,
                   with_weights: bool = True):
    pts = spiral_2d(arms, per_arm, r_max, 0.5)
    mu = voronoi_weights_2d(pts, "disk", r_max + 0.25, 0.4) if with_weights else None
    x0 = phantom_cell_averages(ellipse_phantom_params(phantom_seed), J).astype(np.complex128)
    return pts, mu, x0


def config_c3(J: int = 9, arms: int = 64, per_arm: int = 16384, r_max: float = 256.0,
              with_weights: bool = True):
    pts, mu, x0 = spiral_problem(J, 4, arms, per_arm, r_max, 301, with_weights)
    return {
        "name": "c3", "dim": 2, "J": J, "p": 4, "xi": pts, "mu": mu, "x0": x0,
        "noise_rel": 1e-4, "noise_seed": 302, "tol": 1e-6,
    }


def config_c4_problem(b: int, weights: str = "voronoi"):
    """Problem b (0..63) of the batched workload, seed 4000 + b.

    weights: "voronoi" (cell areas, as C3), "area" (the mean area per point,
    constant: h^2 for the jittered grid, arm gap times arc spacing for the
    spiral -- an O(1) stand-in for the Voronoi areas, which cost tens of
    seconds per million points) or "none"."""
    rng = np.random.default_rng(4000 + b)
    p = int(rng.choice([2, 4]))
    J = int(rng.integers(6, 10))
    pattern = "jitter" if rng.integers(0, 2) == 0 else "spiral"
    M = int(round(rng.uniform(2, 4) * 4 ** J))
    half = 2.0 ** (J - 1)
    if weights not in ("voronoi", "area", "none"):
        raise ValueError(weights)
    if pattern == "jitter":
        pts = jitter_2d(M, half, 4100 + b)
        s = int(round(math.sqrt(M)))
        if weights == "voronoi":
            mu = voronoi_weights_2d(pts, "square", half, 2 * half / math.sqrt(M))
        else:
            mu = np.full(pts.shape[0], (2 * half / s) ** 2) if weights == "area" else None
    else:
        per_arm = max(1, M // 64)
        pts = spiral_2d(64, per_arm, half, 0.5)
        if weights == "voronoi":
            mu = voronoi_weights_2d(pts, "disk", half + 0.25, 0.4)
        else:
            # disk area over the point count = arm gap x arc spacing on average
            mu = np.full(pts.shape[0], math.pi * half * half / pts.shape[0]) if weights == "area" else None
    x0 = phantom_cell_averages(ellipse_phantom_params(4200 + b), J).astype(np.complex128)
    return {"name": f"c4_{b}", "dim": 2, "J": J, "p": p, "pattern": pattern,
            "xi": pts, "mu": mu, "x0": x0, "tol": 1e-6}


def config_c5_pattern(with_weights: bool = True):
    pts = spiral_2d(64, 4096, 128.0, 0.5)
    mu = voronoi_weights_2d(pts, "disk", 128.25, 0.4) if with_weights else None
    return {"name": "c5", "dim": 2, "J": 8, "p": 4, "xi": pts, "mu": mu, "tol": 1e-6}
