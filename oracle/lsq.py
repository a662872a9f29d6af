"""Weighted least-squares solution (Sec. 2, eq. least_squares; Sec. 4.1).

Reading: the weighted problem is argmin_x || W^{1/2} (T x - y) ||_2 with
W = diag(mu); both the data y_m and the rows of T are multiplied by
sqrt(mu_m), as the text of Sec. 4.1 says for the solver.

Reading of "a conjugate gradient procedure" (Sec. 2, Sec. 6): CGLS, i.e.
conjugate gradients on the normal equations A^H A x = A^H b with
A = W^{1/2} T, b = W^{1/2} y, stopped on the relative normal-equation
residual ||A^H (b - A x)|| / ||A^H b||.
"""
from __future__ import annotations

import numpy as np


def lstsq_dense(T: np.ndarray, y: np.ndarray, mu=None) -> np.ndarray:
    """Library solver (LAPACK, SVD based) on the weighted dense system."""
    T = np.asarray(T, complex)
    y = np.asarray(y, complex)
    if mu is not None:
        s = np.sqrt(np.asarray(mu, float))
        T = T * s[:, None]
        y = y * s
    return np.linalg.lstsq(T, y, rcond=None)[0]


def cgls(apply_A, apply_AH, b, x0, tol: float, max_iter: int):
    """Plain CGLS for min ||A x - b||.  Returns (x, iterations, history) where
    history holds the relative normal-equation residual after each iteration."""
    x = np.array(x0, dtype=complex, copy=True)
    r = b - apply_A(x)
    s = apply_AH(r)
    ref = np.linalg.norm(apply_AH(b))
    p = s.copy()
    gamma = np.vdot(s, s).real
    hist = [np.sqrt(gamma) / ref if ref > 0 else 0.0]
    k = 0
    while k < max_iter and np.sqrt(gamma) > tol * ref:
        q = apply_A(p)
        delta = np.vdot(q, q).real
        if delta <= 0:
            break
        alpha = gamma / delta
        x += alpha * p
        r -= alpha * q
        s = apply_AH(r)
        gamma_new = np.vdot(s, s).real
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        k += 1
        hist.append(np.sqrt(gamma) / ref)
    return x, k, np.array(hist)


def normal_residual(apply_A, apply_AH, b, x) -> float:
    ref = np.linalg.norm(apply_AH(b))
    return float(np.linalg.norm(apply_AH(b - apply_A(x))) / ref)
