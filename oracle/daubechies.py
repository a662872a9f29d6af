"""Daubechies low-pass filters and the Fourier transform of the scaling
function, in FP64 (taps derived in 60-digit arithmetic).

Paper passages followed:
* App. A: m0(xi) = sum_k h_k exp(-2 pi i k xi) with m0(0) = 1, and
  F[phi](xi) is the infinite product of m0 over dyadic dilations.
* Sec. 3.3: for p > 1 vanishing moments supp(phi) = [-p+1, p], so the 2p taps
  are indexed k = -p+1 .. p.  Haar (p = 1) is phi = 1_[0,1), taps h_0 = h_1 = 1/2.

Reading (the paper prints no taps and cites the Cohen-Daubechies-Vial filters):
the taps are Daubechies' extremal-phase solution, obtained by spectral
factorization of |m0|^2 = cos^{2p}(pi xi) P(sin^2(pi xi)),
P(y) = sum_{j<p} C(p-1+j, j) y^j, keeping the factor whose zeros in
z = exp(-2 pi i xi) lie outside the unit circle (the larger taps come first).

Reading of the product's start index: the product runs over j >= 1,
F[phi](xi) = prod_{j>=1} m0(2^-j xi).  This is the only start index that
reproduces the Haar closed form printed in App. A; it follows from the
refinement equation phi(x) = 2 sum_k h_k phi(2x - k).
"""
from __future__ import annotations

import functools
import math

import mpmath
import numpy as np

_DPS = 60


@functools.lru_cache(maxsize=None)
def filter_taps_mp(p: int):
    """Taps h_k, k = -p+1..p, as mpmath numbers (60 digits), sum h_k = 1."""
    if p < 1:
        raise ValueError("p must be >= 1")
    with mpmath.workdps(_DPS):
        if p == 1:
            return (mpmath.mpf(1) / 2, mpmath.mpf(1) / 2)
        # P(y) = sum_{j<p} C(p-1+j, j) y^j ; its p-1 roots y_r.
        coeffs = [mpmath.binomial(p - 1 + j, j) for j in range(p)]
        # mpmath.polyroots wants highest degree first
        yroots = mpmath.polyroots(list(reversed(coeffs)), maxsteps=500, extraprec=200)
        if not isinstance(yroots, (list, tuple)):
            yroots = [yroots]
        # sin^2(pi xi) = (2 - z - 1/z)/4 with z = exp(-2 pi i xi); each y_r gives
        # z^2 - 2(1 - 2 y_r) z + 1 = 0, roots z and 1/z.  Keep |z| > 1.
        zroots = []
        for y in yroots:
            b = 1 - 2 * y
            s = mpmath.sqrt(b * b - 1)
            z1, z2 = b + s, b - s
            zroots.append(z1 if abs(z1) > 1 else z2)
        # polynomial in z: ((1+z)/2)^p * prod (z - z_r), coefficients ascending
        poly = [mpmath.mpc(1)]
        for _ in range(p):
            poly = _polymul(poly, [mpmath.mpc(1) / 2, mpmath.mpc(1) / 2])
        for zr in zroots:
            poly = _polymul(poly, [-zr, mpmath.mpc(1)])
        total = mpmath.fsum(poly)
        taps = [mpmath.re(c / total) for c in poly]
        return tuple(taps)


def _polymul(a, b):
    out = [mpmath.mpc(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def filter_taps(p: int) -> np.ndarray:
    """FP64 taps h_k for k = -p+1 .. p (array index k + p - 1)."""
    return np.array([float(t) for t in filter_taps_mp(p)], dtype=np.float64)


def tap_indices(p: int) -> np.ndarray:
    return np.arange(-p + 1, p + 1)


def m0(xi, p: int, taps: np.ndarray | None = None) -> np.ndarray:
    """Low-pass filter m0(xi) = sum_k h_k exp(-2 pi i k xi) (App. A)."""
    h = filter_taps(p) if taps is None else taps
    k = np.arange(-p + 1, -p + 1 + len(h))
    xi = np.asarray(xi, dtype=np.float64)
    # sum_k h_k = 1 exactly (App. A normalization), so
    # m0 = 1 + sum_k h_k (exp(-2 pi i k xi) - 1), with exp(i t) - 1 = 2i sin(t/2) exp(i t/2)
    # evaluated without cancellation; this keeps m0(0) = 1 exact in FP64.
    t = -2.0 * np.pi * np.multiply.outer(xi, k)
    em1 = 2j * np.sin(0.5 * t) * np.exp(0.5j * t)
    return 1.0 + em1 @ h


def product_depth(xi) -> int:
    """Number of factors kept in the infinite product: 60 + ceil(log2 max|xi|),
    so that the omitted tail F[phi](2^-K xi) - 1 = O(2^-K |xi|) is below FP64
    rounding."""
    mx = float(np.max(np.abs(xi))) if np.size(xi) else 0.0
    return 60 + max(0, math.ceil(math.log2(mx))) if mx > 1 else 60


def phi_hat(xi, p: int, depth: int | None = None, taps: np.ndarray | None = None) -> np.ndarray:
    """F[phi](xi) = prod_{j=1}^{K} m0(2^-j xi)  (App. A)."""
    xi = np.asarray(xi, dtype=np.float64)
    K = product_depth(xi) if depth is None else depth
    out = np.ones(xi.shape, dtype=np.complex128)
    for j in range(1, K + 1):
        out *= m0(xi / 2.0 ** j, p, taps)
    return out


def phi_hat_suffix(xi, p: int, depth: int, taps: np.ndarray | None = None) -> np.ndarray:
    """All dilates F[phi](xi / 2^l) for l = 0..depth, as an array of shape
    (depth+1, *xi.shape), each the product prod_{j>l} m0(2^-j xi) truncated at
    j = depth + 60 (the tail below l is the same product started later)."""
    xi = np.asarray(xi, dtype=np.float64)
    top = depth + 60
    fac = np.empty((top,) + xi.shape, dtype=np.complex128)
    for j in range(1, top + 1):
        fac[j - 1] = m0(xi / 2.0 ** j, p, taps)
    suffix = np.empty((depth + 1,) + xi.shape, dtype=np.complex128)
    acc = np.ones(xi.shape, dtype=np.complex128)
    # suffix[l] = prod_{j=l+1}^{top} fac[j-1]
    for j in range(top, 0, -1):
        acc = acc * fac[j - 1]
        l = j - 1
        if l <= depth:
            suffix[l] = acc
    return suffix


def haar_phi_hat_closed_form(xi) -> np.ndarray:
    """App. A closed form for Haar: (1 - exp(-2 pi i xi)) / (2 pi i xi), 1 at 0."""
    xi = np.asarray(xi, dtype=np.float64)
    out = np.ones(xi.shape, dtype=np.complex128)
    nz = xi != 0
    out[nz] = (1 - np.exp(-2j * np.pi * xi[nz])) / (2j * np.pi * xi[nz])
    return out
