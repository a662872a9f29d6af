"""Cohen-Daubechies-Vial boundary scaling functions and the Fourier transform
of the left/right boundary functions (App. A.1 of the paper).

The paper uses the boundary functions of Cohen, Daubechies and Vial but
prints neither their filters H, h nor their construction.  This module
derives them from the defining properties, in 60-digit arithmetic:

1. Edge space (half-line [0, inf), scale 0).  Polynomials of degree < p on
   [0, inf) are sum_n c_j(n) phi(x - n) restricted to x >= 0, with c_j a
   polynomial of degree j in n.  Translates n >= p lie inside (0, inf) and
   stay interior; the restricted translates n = -p+1 .. p-1 carry the rest, so
   the edge space is E = { sum_{n=-p+1}^{p-1} P(n) phi(x-n) 1_{x>=0} : deg P < p }.
   Every element of E is orthogonal to the interior translates.
2. Truncated Gram matrix G[n,n'] = int_0^inf phi(x-n) phi(x-n') dx.  It is
   delta when either translate lies in [0, inf) (n >= p-1), zero when either
   lies in (-inf, 0] (n <= -p); the remaining entries solve the refinement
   identity G[n,n'] = 2 sum_{k,k'} h_k h_k' G[2n+k, 2n'+k'].
3. Staircase: phi^L_k lies in E and uses translates n <= k only (support
   [0, p+k], which is the sparsity pattern of V printed in App. A.1); the
   functions are made orthonormal in the order k = 0, 1, ..., p-1.
   Reading (sign, unpinned by the paper): the coefficient of translate n = k
   is positive.
4. Filters from the left dilation equation of App. A.1,
   (1/sqrt2) phi^L_k(x) = sum_l H_kl phi^L_l(2x) + sum_{m=p}^{p+2k} h_km phi(2x-m):
   H_kl = sqrt2 <phi^L_k, phi^L_l(2.)>,  h_km = sqrt2 <phi^L_k, phi(2.-m)>.
5. U = H/sqrt2, V = h/sqrt2 (columns m = p..3p-2); v1(0) solves
   v1(0) = U v1(0) + V v2(0) with v2(0) = (1,..,1) because F[phi](0) = 1.
6. v1(xi) = U^K v1(0) + sum_{l<K} U^l V v2(xi / 2^(l+1)) (App. A.1).

Right edge (reading of "completely analogous"): reflect.  With the flipped
filter h^b_k = h_{1-k} (same index range), phi^b(x) = phi(1-x); build the left
functions of phi^b and set phi^R_k(x) = phi^bL_k(-x).  This reproduces the
printed right dilation equation with phi(2x+m+1) exactly, and
v2^R(xi) = [F[phi](xi) exp(2 pi i (m+1) xi)]_{m=p}^{3p-2} as printed.
"""
from __future__ import annotations

import functools
import math

import mpmath
import numpy as np

from . import daubechies as db

_DPS = 60


def _gram_solver(h_mp, p):
    """Return G(n, n') for all integers as mpmath numbers (half-line Gram)."""
    lo, hi = -p + 1, p - 2           # unknown range (both indices)
    idx = [(n, m) for n in range(lo, hi + 1) for m in range(n, hi + 1)]
    pos = {pair: i for i, pair in enumerate(idx)}
    nu = len(idx)
    kk = list(range(-p + 1, p + 1))

    def known(n, m):
        if n >= p - 1 or m >= p - 1:
            return mpmath.mpf(1) if n == m else mpmath.mpf(0)
        if n <= -p or m <= -p:
            return mpmath.mpf(0)
        return None

    with mpmath.workdps(_DPS):
        A = mpmath.zeros(nu, nu)
        b = mpmath.zeros(nu, 1)
        for (n, m), row in pos.items():
            A[row, row] += 1
            for ia, ka in enumerate(kk):
                for ib, kb in enumerate(kk):
                    coef = 2 * h_mp[ia] * h_mp[ib]
                    s, t = 2 * n + ka, 2 * m + kb
                    val = known(s, t)
                    if val is None:
                        key = (s, t) if s <= t else (t, s)
                        A[row, pos[key]] -= coef
                    else:
                        b[row] += coef * val
        sol = mpmath.qr_solve(A, b)[0] if nu > 0 else []
        resid = mpmath.norm(A * sol - b) if nu > 0 else mpmath.mpf(0)

    table = {pair: sol[i] for i, pair in enumerate(idx)}

    def G(n, m):
        v = known(n, m)
        if v is not None:
            return v
        return table[(n, m) if n <= m else (m, n)]

    return G, resid


class EdgeConstruction:
    """Left-edge CDV construction for a filter with taps on k = -p+1..p."""

    def __init__(self, h_mp, p):
        self.p = p
        self.h_mp = list(h_mp)
        with mpmath.workdps(_DPS):
            self.G, self.gram_residual = _gram_solver(self.h_mp, p)
            self.trans = list(range(-p + 1, p))            # translates n of E
            self.coef = self._staircase()                   # p x (2p-1) mp
            self.H, self.h, self.refined = self._filters()

    def inner(self, a, b):
        """<sum a_n phi(.-n)1, sum b_n phi(.-n)1> over n in self.trans."""
        tot = mpmath.mpf(0)
        for i, n in enumerate(self.trans):
            if a[i] == 0:
                continue
            for j, m in enumerate(self.trans):
                if b[j] == 0:
                    continue
                tot += a[i] * b[j] * self.G(n, m)
        return tot

    def _staircase(self):
        p = self.p
        basis = []
        for k in range(p):
            v = []
            for n in self.trans:
                val = mpmath.mpf(1)
                for t in range(k + 1, p):
                    val *= (n - t)
                v.append(val)
            for prev in basis:
                c = self.inner(v, prev)
                v = [x - c * y for x, y in zip(v, prev)]
            nrm = mpmath.sqrt(self.inner(v, v))
            v = [x / nrm for x in v]
            if v[self.trans.index(k)] < 0:
                v = [-x for x in v]
            basis.append(v)
        return basis

    def _filters(self):
        p = self.p
        kk = list(range(-p + 1, p + 1))
        s_lo, s_hi = 2 * (-p + 1) + (-p + 1), 2 * (p - 1) + p
        refined = []
        for k in range(p):
            bs = {}
            for i, n in enumerate(self.trans):
                a = self.coef[k][i]
                if a == 0:
                    continue
                for j, t in enumerate(kk):
                    s = 2 * n + t
                    bs[s] = bs.get(s, mpmath.mpf(0)) + 2 * a * self.h_mp[j]
            refined.append(bs)
        r2 = mpmath.sqrt(2)
        H = mpmath.zeros(p, p)
        hh = mpmath.zeros(p, 2 * p - 1)              # columns m = p .. 3p-2
        for k in range(p):
            for l in range(p):
                tot = mpmath.mpf(0)
                for s, bv in refined[k].items():
                    for j, t in enumerate(self.trans):
                        a = self.coef[l][j]
                        if a != 0:
                            tot += bv * a * self.G(s, t)
                H[k, l] = tot / r2
            for mi, m in enumerate(range(p, 3 * p - 1)):
                tot = mpmath.mpf(0)
                for s, bv in refined[k].items():
                    tot += bv * self.G(s, m)
                hh[k, mi] = tot / r2
        return H, hh, refined

    # --- FP64 exports -------------------------------------------------
    def U(self):
        return np.array([[float(self.H[i, j]) / math.sqrt(2) for j in range(self.p)]
                         for i in range(self.p)])

    def V(self):
        return np.array([[float(self.h[i, j]) / math.sqrt(2) for j in range(2 * self.p - 1)]
                         for i in range(self.p)])

    def v1_zero(self):
        """Solve v1(0) = U v1(0) + V 1 (App. A.1, xi = 0) in 60 digits."""
        with mpmath.workdps(_DPS):
            p = self.p
            r2 = mpmath.sqrt(2)
            A = mpmath.eye(p) - self.H / r2
            rhs = mpmath.matrix([sum(self.h[i, j] for j in range(2 * p - 1)) / r2 for i in range(p)])
            sol = mpmath.qr_solve(A, rhs)[0]
            return np.array([float(sol[i]) for i in range(p)])

    def integrals(self):
        """int_0^inf phi^L_k = sum_n a_n sum_n' G[n,n'] (partition of unity);
        an independent route to v1(0)."""
        with mpmath.workdps(_DPS):
            out = []
            for k in range(self.p):
                tot = mpmath.mpf(0)
                for i, n in enumerate(self.trans):
                    for m in range(-self.p + 1, self.p):
                        tot += self.coef[k][i] * self.G(n, m)
                out.append(float(tot))
            return np.array(out)

    def coef_fp64(self):
        return np.array([[float(x) for x in row] for row in self.coef])


@functools.lru_cache(maxsize=None)
def left_edge(p: int) -> EdgeConstruction:
    if p < 2:
        raise ValueError("boundary functions exist for p >= 2 only")
    return EdgeConstruction(db.filter_taps_mp(p), p)


@functools.lru_cache(maxsize=None)
def flipped_edge(p: int) -> EdgeConstruction:
    """Left construction for the reflected filter h^b_k = h_{1-k}; its H, h are
    the right-edge filters."""
    if p < 2:
        raise ValueError("boundary functions exist for p >= 2 only")
    h = db.filter_taps_mp(p)           # index k + p - 1
    flipped = [h[(1 - k) + p - 1] for k in range(-p + 1, p + 1)]
    return EdgeConstruction(flipped, p)


def _recursion(xi, p, U, V, v1_0, sign):
    """v1(xi) by the truncated dilation recursion.  sign=-1: left edge,
    v2(z)_m = F[phi](z) exp(-2 pi i m z); sign=+1: right edge,
    v2(z)_m = F[phi](z) exp(+2 pi i (m+1) z); m = p..3p-2."""
    xi = np.asarray(xi, dtype=np.float64)
    flat = xi.reshape(-1)
    K = db.product_depth(flat)
    sfx = db.phi_hat_suffix(flat, p, K)          # sfx[l] = F[phi](xi / 2^l)
    ms = np.arange(p, 3 * p - 1)
    shift = ms + (1 if sign > 0 else 0)
    w = np.repeat(v1_0[:, None].astype(np.complex128), flat.size, axis=1)
    for l in range(K - 1, -1, -1):
        z = flat / 2.0 ** (l + 1)
        v2 = sfx[l + 1][None, :] * np.exp(sign * 2j * np.pi * np.multiply.outer(shift, z))
        w = U @ w + V @ v2
    return w.reshape((p,) + xi.shape)


def left_phi_hat(xi, p: int) -> np.ndarray:
    """[F[phi^L_k](xi)]_{k=0}^{p-1}, shape (p, *xi.shape)."""
    e = left_edge(p)
    return _recursion(xi, p, e.U(), e.V(), e.v1_zero(), -1)


def right_phi_hat(xi, p: int) -> np.ndarray:
    """[F[phi^R_k](xi)]_{k=0}^{p-1}, shape (p, *xi.shape)."""
    e = flipped_edge(p)
    return _recursion(xi, p, e.U(), e.V(), e.v1_zero(), +1)
