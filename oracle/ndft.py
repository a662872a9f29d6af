"""Non-uniform discrete Fourier transform by direct sums (Sec. 3.2).

y_m = sum_{k in I_N} x_k exp(-2 pi i k . xi_m), I_N = Z^D cap prod [-N_d/2, N_d/2),
and the adjoint z_k = sum_m y_m exp(+2 pi i k . xi_m).  Coefficient arrays are
indexed by k + N/2 along every axis.
"""
from __future__ import annotations

import mpmath
import numpy as np


def _phase(xi, k, sign):
    """exp(sign 2 pi i xi k), argument reduced mod 1 in extended precision."""
    t = np.multiply.outer(np.asarray(xi, np.float64).astype(np.longdouble), np.asarray(k, np.longdouble))
    return np.exp(sign * 2j * np.pi * (t - np.round(t)).astype(np.float64))


def ndft_1d(x, xi):
    N = len(x)
    k = np.arange(-N // 2, N // 2)
    return _phase(xi, k, -1.0) @ np.asarray(x, complex)


def ndft_adjoint_1d(y, xi, N):
    k = np.arange(-N // 2, N // 2)
    return _phase(xi, k, +1.0).T @ np.asarray(y, complex)


def ndft_2d(X, xi2):
    """X of shape (N1, N2), xi2 of shape (M, 2)."""
    N1, N2 = X.shape
    k1 = np.arange(-N1 // 2, N1 // 2)
    k2 = np.arange(-N2 // 2, N2 // 2)
    xi2 = np.asarray(xi2, float)
    E1 = _phase(xi2[:, 0], k1, -1.0)     # (M, N1)
    E2 = _phase(xi2[:, 1], k2, -1.0)     # (M, N2)
    return np.einsum("mi,ij,mj->m", E1, np.asarray(X, complex), E2)


def ndft_adjoint_2d(y, xi2, N1, N2):
    k1 = np.arange(-N1 // 2, N1 // 2)
    k2 = np.arange(-N2 // 2, N2 // 2)
    xi2 = np.asarray(xi2, float)
    E1 = _phase(xi2[:, 0], k1, +1.0).T   # (N1, M)
    E2 = _phase(xi2[:, 1], k2, +1.0)     # (M, N2)
    return E1 @ (np.asarray(y, complex)[:, None] * E2)


def ndft_1d_mp(x, xi, dps=40):
    """Tiny-case NDFT in mpmath (for pinning the FP64 sums)."""
    N = len(x)
    with mpmath.workdps(dps):
        out = []
        for xm in xi:
            s = mpmath.mpc(0)
            for idx, k in enumerate(range(-N // 2, N // 2)):
                s += mpmath.mpc(complex(x[idx])) * mpmath.expj(-2 * mpmath.pi * k * mpmath.mpf(float(xm)))
            out.append(complex(s))
    return np.array(out)
