"""Scaling functions in space, on dyadic grids, from the refinement equation
phi(x) = 2 sum_k h_k phi(2x - k) (App. A; Sec. 3.3), and numerical Fourier
transforms of them.

Used only as an independent pin for the Fourier-side routines: nothing here
shares a step with the infinite product or the dilation recursion.

Values at the integers come from the eigenvector of the refinement equation
restricted to the integers (eigenvalue 1, normalized by partition of unity);
values at x = j / 2^R then follow level by level from the refinement
equation.
"""
from __future__ import annotations

import numpy as np

from . import daubechies as db


def phi_on_grid(p: int, R: int, taps: np.ndarray | None = None):
    """(x, phi(x)) for x = j / 2^R covering supp phi = [-p+1, p]."""
    h = db.filter_taps(p) if taps is None else np.asarray(taps, float)
    lo, hi = -p + 1, p
    if p == 1:
        x = np.arange(0, 2 ** R + 1) / 2 ** R
        v = np.where(x < 1, 1.0, 0.0)
        return x, v
    ints = np.arange(lo, hi + 1)
    n = len(ints)
    A = np.zeros((n, n))
    for a, i in enumerate(ints):
        for b, j in enumerate(ints):
            k = 2 * i - j
            if lo <= k <= hi:
                A[a, b] = 2 * h[k - lo]
    w, V = np.linalg.eig(A)
    e = np.argmin(np.abs(w - 1))
    vals = np.real(V[:, e])
    vals = vals / vals.sum()
    # level by level: grid spacing 2^-r
    grid = {i: vals[a] for a, i in enumerate(ints)}    # keys: integer numerators at level r
    cur = np.array([grid[i] for i in ints])
    cur_lo = lo
    for r in range(1, R + 1):
        # new grid numerators j at spacing 2^-r: j in [lo*2^r, hi*2^r]
        js = np.arange(lo * 2 ** r, hi * 2 ** r + 1)
        out = np.zeros(js.size)
        # phi(j/2^r) = 2 sum_k h_k phi(j/2^(r-1) - k) ; previous level spacing 2^-(r-1)
        for kk in range(lo, hi + 1):
            num = js - kk * 2 ** (r - 1)                      # numerator at level r-1
            valid = (num >= cur_lo) & (num < cur_lo + cur.size)
            out[valid] += 2 * h[kk - lo] * cur[num[valid] - cur_lo]
        cur = out
        cur_lo = lo * 2 ** r
    x = np.arange(cur_lo, cur_lo + cur.size) / 2 ** R
    return x, cur


def eval_translates(x_grid, phi_vals, R, x, n):
    """phi(x - n) for x on the same dyadic grid (exact lookup)."""
    step = 2 ** R
    base = int(round(x_grid[0] * step))
    idx = np.rint((np.asarray(x) - n) * step).astype(np.int64) - base
    out = np.zeros(np.shape(x))
    ok = (idx >= 0) & (idx < phi_vals.size)
    out[ok] = phi_vals[idx[ok]]
    return out


def trapezoid_ft(x, f, xi):
    """Trapezoid rule for int f(x) exp(-2 pi i xi x) dx on a uniform grid."""
    hstep = x[1] - x[0]
    wts = np.full(x.size, hstep)
    wts[0] = wts[-1] = hstep / 2
    return np.exp(-2j * np.pi * np.multiply.outer(np.asarray(xi, float), x)) @ (wts * f)


def trapezoid_inner(x, f, g):
    hstep = x[1] - x[0]
    wts = np.full(x.size, hstep)
    wts[0] = wts[-1] = hstep / 2
    return float(np.sum(wts * f * g))


def basis_on_grid(J: int, p: int, R: int):
    """(x, S) with x_j = -1/2 + j / 2^R (j = 0..2^R) and S[n, j] = s_n(x_j), the
    basis of V_J^int on [-1/2, 1/2] (Sec. 3.3) in space, R >= J:
      n <  p      : 2^{J/2} phi^L_n(2^J (x + 1/2))
      p <= n < N-p: 2^{J/2} phi(2^J (x + 1/2) - n)
      n >= N-p    : 2^{J/2} phi^R_{N-1-n}(2^J (x - 1/2))
    The boundary functions are the restricted combinations of translates that
    define them (App. A.1): phi^L_k(t) = sum_i a_{k,i} phi(t - n_i) for t >= 0,
    and phi^R_k(t) = phi^{bL}_k(-t) for t <= 0, where the reflected filter
    h_{1-k} has the scaling function phi(1 - t).  phi comes from the cascade at
    resolution r = R - J, so every needed value is read at a grid point."""
    from . import cdv
    if R < J:
        raise ValueError("need R >= J")
    r = R - J
    N = 1 << J
    xg, ph = phi_on_grid(p, r)
    t = np.arange(2 ** R + 1) / 2 ** r                # t = 2^J (x + 1/2) in [0, N]
    S = np.zeros((N, t.size))
    nb = 0 if p == 1 else p
    for n in range(nb, N - nb):
        S[n] = eval_translates(xg, ph, r, t, n)
    if nb:
        eL, eR = cdv.left_edge(p), cdv.flipped_edge(p)
        A, B = eL.coef_fp64(), eR.coef_fp64()
        u = t - N                                       # <= 0 on the whole interval
        for k in range(p):
            S[k] = sum(A[k, i] * eval_translates(xg, ph, r, t, n) for i, n in enumerate(eL.trans))
            S[N - 1 - k] = sum(B[k, i] * eval_translates(xg, ph, r, 1 + u + n, 0) for i, n in enumerate(eR.trans))
    return t / N - 0.5, 2.0 ** (J / 2) * S


def weval(coefs, J: int, p: int, R: int):
    """f = sum_n x_n s_n on the dyadic grid x_j = -1/2 + j / 2^R (1D), or
    f(x_a, y_b) = sum_{i,j} X[i, j] s_i(x_a) s_j(y_b) (2D, X row-major with i
    the x index): the weval of Sec. 6.2."""
    c = np.asarray(coefs)
    x, S = basis_on_grid(J, p, R)
    if c.ndim == 1:
        return x, c @ S
    return x, S.T @ c @ S
