"""Dense change-of-basis matrix T (Sec. 4 for 1D, Sec. 5 and App. C for 2D).

Entry T[m, n] = F[phi^int_{J, n-N/2}](xi_m) for the boundary-corrected basis of
V_J^int on [-1/2, 1/2] (Sec. 3.3), N = 2^J, with 0-based column n:

  n <  p        : 2^{-J/2} exp(+i pi xi) F[phi^L_n](2^-J xi)
  p <= n < N-p  : 2^{-J/2} exp(-2 pi i (n - N/2) 2^-J xi) F[phi](2^-J xi)
  n >= N-p      : 2^{-J/2} exp(-i pi xi) F[phi^R_{N-1-n}](2^-J xi)

(Sec. 4 and the Fourier dilation/translation rules of App. A.)  Readings of
garbled passages in Sec. 4: the interior phase carries the factor 2 of the
general translation rule; the boundary translates are by -1/2 and +1/2 as in
the definition of phi^int (the printed phases exp(+-i pi xi) agree); the
interior column of 1-based index n has translation n-1-2^{J-1}.  For Haar
(p = 1) every column is interior.

2D (Sec. 5, App. C): T[m, (i, j)] = b_i(xi_x,m) b_j(xi_y,m), i.e. each row is
the Kronecker product of the two 1D rows.  Coefficients are stored row-major
X[i, j] with i the x index, so vec(X)[i*N + j] = X[i, j].
"""
from __future__ import annotations

import numpy as np

from . import cdv
from . import daubechies as db


def unit_phase(k, eta, sign: float = -1.0) -> np.ndarray:
    """exp(sign 2 pi i k eta) as an outer product over integer k and real eta.
    The argument k*eta is reduced modulo 1 in x87 extended precision before the
    exponential: in plain FP64 the product k*eta ~ N/2 carries an absolute
    rounding error ~ 1e-11 at N = 16384."""
    kk = np.asarray(k, dtype=np.longdouble)
    ee = np.asarray(eta, dtype=np.float64).astype(np.longdouble)
    t = np.multiply.outer(kk, ee)
    frac = (t - np.round(t)).astype(np.float64)
    return np.exp(sign * 2j * np.pi * frac)


def half_turn_phase(xi, sign: float) -> np.ndarray:
    """exp(sign i pi xi) with the exact reduction xi mod 2."""
    r = np.fmod(np.asarray(xi, dtype=np.float64), 2.0)
    return np.exp(sign * 1j * np.pi * r)


def n_boundary(p: int) -> int:
    return 0 if p == 1 else p


def check_scale(J: int, p: int):
    if (1 << J) < 2 * p:
        raise ValueError("need 2^J >= 2p")


def columns_1d(xi, J: int, p: int) -> np.ndarray:
    """B[n, m] = b_n(xi_m), shape (N, M): all 1D columns at the given points."""
    check_scale(J, p)
    xi = np.asarray(xi, dtype=np.float64)
    N = 1 << J
    eta = xi / N
    scale = 2.0 ** (-J / 2.0)
    B = np.empty((N, xi.size), dtype=np.complex128)
    ph = db.phi_hat(eta, p)
    nb = n_boundary(p)
    k = np.arange(nb, N - nb) - N // 2
    B[nb:N - nb] = scale * unit_phase(k, eta, -1.0) * ph[None, :]
    if nb:
        L = cdv.left_phi_hat(eta, p)                 # (p, M)
        R = cdv.right_phi_hat(eta, p)
        B[:nb] = scale * half_turn_phase(xi, +1.0)[None, :] * L
        # column N-1-k holds phi^R_k
        B[N - nb:] = (scale * half_turn_phase(xi, -1.0)[None, :] * R)[::-1]
    return B


def column_1d(xi, J: int, p: int, n: int) -> np.ndarray:
    """b_n(xi_m) for a single column n: the formulas of columns_1d for that
    column only (Sec. 4), so that one coefficient of T^H u can be formed over
    many points without building every column."""
    check_scale(J, p)
    xi = np.asarray(xi, dtype=np.float64)
    N = 1 << J
    if not 0 <= n < N:
        raise ValueError("column index out of range")
    eta = xi / N
    scale = 2.0 ** (-J / 2.0)
    nb = n_boundary(p)
    if nb <= n < N - nb:
        return scale * unit_phase([n - N // 2], eta, -1.0)[0] * db.phi_hat(eta, p)
    if n < nb:
        return scale * half_turn_phase(xi, +1.0) * cdv.left_phi_hat(eta, p)[n]
    return scale * half_turn_phase(xi, -1.0) * cdv.right_phi_hat(eta, p)[N - 1 - n]


def columns_subset_1d(xi, J: int, p: int, ns) -> dict:
    """{n: b_n(xi)} for the listed columns n, by the formulas of columns_1d
    (Sec. 4), with phi-hat and the boundary transforms evaluated once for all
    requested columns rather than once per column."""
    check_scale(J, p)
    xi = np.asarray(xi, dtype=np.float64)
    N = 1 << J
    eta = xi / N
    scale = 2.0 ** (-J / 2.0)
    nb = n_boundary(p)
    ns = sorted(set(int(n) for n in ns))
    if any(not 0 <= n < N for n in ns):
        raise ValueError("column index out of range")
    out = {}
    inner = [n for n in ns if nb <= n < N - nb]
    if inner:
        ph = db.phi_hat(eta, p)
        for n in inner:
            out[n] = scale * unit_phase([n - N // 2], eta, -1.0)[0] * ph
    if any(n < nb for n in ns):
        L = cdv.left_phi_hat(eta, p)
        for n in (n for n in ns if n < nb):
            out[n] = scale * half_turn_phase(xi, +1.0) * L[n]
    if any(n >= N - nb for n in ns):
        R = cdv.right_phi_hat(eta, p)
        for n in (n for n in ns if n >= N - nb):
            out[n] = scale * half_turn_phase(xi, -1.0) * R[N - 1 - n]
    return out


def dense_T_1d(xi, J: int, p: int) -> np.ndarray:
    """T of shape (M, N), 1D."""
    return columns_1d(xi, J, p).T.copy()


def dense_T_2d(xi2, J: int, p: int) -> np.ndarray:
    """T of shape (M, N*N) for 2D points xi2 of shape (M, 2); row m is
    kron(b(xi_x,m), b(xi_y,m)) (App. C).  Small sizes only."""
    xi2 = np.asarray(xi2, dtype=np.float64)
    Bx = columns_1d(xi2[:, 0], J, p)
    By = columns_1d(xi2[:, 1], J, p)
    M = xi2.shape[0]
    N = 1 << J
    T = np.empty((M, N * N), dtype=np.complex128)
    for m in range(M):
        T[m] = np.kron(Bx[:, m], By[:, m])
    return T


def apply_T_2d(xi2, J: int, p: int, X: np.ndarray, chunk: int = 16384) -> np.ndarray:
    """y_m = sum_{i,j} b_i(xi_x) X[i,j] b_j(xi_y), through per-dimension dense
    columns and a matrix product (no M x N^2 matrix is formed)."""
    xi2 = np.asarray(xi2, dtype=np.float64)
    X = np.asarray(X, dtype=np.complex128)
    M = xi2.shape[0]
    y = np.empty(M, dtype=np.complex128)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        Bx = columns_1d(xi2[s:e, 0], J, p)       # (N, c)
        By = columns_1d(xi2[s:e, 1], J, p)
        y[s:e] = np.einsum("im,im->m", Bx, X @ By)
    return y


def apply_TH_2d(xi2, J: int, p: int, u: np.ndarray, chunk: int = 16384) -> np.ndarray:
    """X[i,j] = sum_m conj(b_i(xi_x,m)) conj(b_j(xi_y,m)) u_m (adjoint, App. C)."""
    xi2 = np.asarray(xi2, dtype=np.float64)
    u = np.asarray(u, dtype=np.complex128)
    N = 1 << J
    X = np.zeros((N, N), dtype=np.complex128)
    for s in range(0, xi2.shape[0], chunk):
        e = min(xi2.shape[0], s + chunk)
        Bx = columns_1d(xi2[s:e, 0], J, p)
        By = columns_1d(xi2[s:e, 1], J, p)
        X += np.conj(Bx) @ (u[s:e, None] * np.conj(By).T)
    return X


def apply_T_1d(xi, J: int, p: int, x: np.ndarray, chunk: int = 16384) -> np.ndarray:
    xi = np.asarray(xi, dtype=np.float64)
    y = np.empty(xi.size, dtype=np.complex128)
    for s in range(0, xi.size, chunk):
        e = min(xi.size, s + chunk)
        y[s:e] = columns_1d(xi[s:e], J, p).T @ x
    return y


def apply_TH_1d(xi, J: int, p: int, u: np.ndarray, chunk: int = 16384) -> np.ndarray:
    xi = np.asarray(xi, dtype=np.float64)
    N = 1 << J
    x = np.zeros(N, dtype=np.complex128)
    for s in range(0, xi.size, chunk):
        e = min(xi.size, s + chunk)
        x += np.conj(columns_1d(xi[s:e], J, p)) @ u[s:e]
    return x


def rows_T_2d(xi2, J: int, p: int, X: np.ndarray, rows) -> np.ndarray:
    """Selected outputs y_m of the 2D forward product, one by one."""
    rows = np.asarray(rows)
    return apply_T_2d(np.asarray(xi2)[rows], J, p, X)


def coeffs_TH_2d(xi2, J: int, p: int, u: np.ndarray, ij, chunk: int = 65536) -> np.ndarray:
    """Selected adjoint outputs X[i,j] = sum_m conj(b_i(xi_x,m) b_j(xi_y,m)) u_m."""
    xi2 = np.asarray(xi2, dtype=np.float64)
    ij = np.asarray(ij)
    ii = np.unique(ij[:, 0])
    jj = np.unique(ij[:, 1])
    out = np.zeros(len(ij), dtype=np.complex128)
    for s in range(0, xi2.shape[0], chunk):
        e = min(xi2.shape[0], s + chunk)
        Bx = columns_1d(xi2[s:e, 0], J, p)
        By = columns_1d(xi2[s:e, 1], J, p)
        cx = {i: np.conj(Bx[i]) for i in ii}
        cy = {j: np.conj(By[j]) for j in jj}
        for q, (i, j) in enumerate(ij):
            out[q] += np.sum(cx[i] * cy[j] * u[s:e])
    return out
