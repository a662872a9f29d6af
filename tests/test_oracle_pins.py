"""Pins for the FP64 oracle: each check is fixed by the paper, by a closed
form, by an invariant of the mathematics, or by an independent route (space
domain, library FFT, arbitrary precision), never by re-typing the oracle's
own formula."""
import math
import os

import numpy as np
import pytest

from oracle import basis, cascade, cdv, lsq, ndft
from oracle import daubechies as db

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=", 1)
                vals[k.strip()] = [float(eval(t, {"sqrt": math.sqrt})) for t in v.split(",")]
    return vals


# ---------------------------------------------------------------- filters (O1)

def test_db2_taps_closed_form():
    g = _golden("db2_taps.txt")
    assert np.allclose(db.filter_taps(2), g["h"], rtol=0, atol=3e-16)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_filter_invariants(p):
    h = db.filter_taps(p)
    k = db.tap_indices(p).astype(float)
    assert len(h) == 2 * p
    assert abs(h.sum() - 1) < 1e-15                           # m0(0) = 1 (App. A)
    for j in range(p):                                         # m0 has a zero of order p at 1/2
        assert abs(np.sum((-1) ** k * (k / p) ** j * h)) < 1e-14
    for l in range(1, p):                                      # orthonormal translates
        assert abs(np.dot(h[:-2 * l], h[2 * l:])) < 1e-15
    assert abs(np.dot(h, h) - 0.5) < 1e-15
    if p > 1:                                                   # extremal phase: larger taps first
        assert abs(h[0]) > abs(h[-1])


def test_db4_taps_textbook_table():
    """db4 (p = 4) against Daubechies' published extremal-phase table (Ten
    Lectures, Table 6.1, N = 4), which fixes the phase family that the
    invariants above leave open."""
    g = _golden("db4_taps.txt")
    want = np.array(g["h_sqrt2"]) / math.sqrt(2.0)
    # the table prints 16 decimals (+-5e-17); FP64 spacing near 0.5 is 1.1e-16
    assert np.max(np.abs(db.filter_taps(4) - want)) < 3e-16


def _zeros_off_minus_one(h, p):
    """Zeros of the polynomial sum_k h_k z^(k+p-1) other than the p-fold
    zero at z = -1, found by dividing ((1+z)/2)^p out of the coefficients."""
    lead_first = np.asarray(h, dtype=float)[::-1]
    q, r = np.polydiv(lead_first, np.poly1d([0.5, 0.5]) ** p)
    assert np.max(np.abs(r)) < 1e-13          # the p-fold zero at z = -1 is there
    return np.roots(q)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_filter_zero_locations(p):
    """Extremal phase: with z = exp(-2 pi i xi), every zero of m0 apart from
    z = -1 lies strictly outside the unit circle (the factor of
    |m0|^2 = cos^{2p}(pi xi) P(sin^2 pi xi) that keeps the outer roots).  A
    filter of another phase family (least asymmetric, or any mix) has zeros on
    both sides and fails here."""
    z = _zeros_off_minus_one(db.filter_taps(p), p)
    assert len(z) == p - 1
    assert np.min(np.abs(z)) > 1.5


def _reflected_pair_taps(p):
    """Another real orthonormal filter with the same |m0|: the oracle's taps
    with one complex-conjugate pair of zeros z, conj(z) moved to 1/conj(z), 1/z
    (a planted phase mistake, used only to show the pins reject it)."""
    h = db.filter_taps(p)
    z = _zeros_off_minus_one(h, p)
    k = int(np.argmax(np.abs(z.imag)))
    assert abs(z[k].imag) > 1e-3
    pair = [z[k], np.conj(z[k])]
    rest = [w for i, w in enumerate(z) if not (np.isclose(w, pair[0]) or np.isclose(w, pair[1]))]
    new = rest + [1 / np.conj(pair[0]), 1 / np.conj(pair[1])]
    poly = np.poly1d([0.5, 0.5]) ** p * np.poly1d(np.poly(new))
    c = np.real(poly.coeffs[::-1])
    return c / c.sum()


@pytest.mark.parametrize("p", [3, 4, 6])
def test_phase_pins_reject_other_factorizations(p):
    """The planted filter passes every invariant of test_filter_invariants
    (sum, vanishing moments, double-shift orthonormality) but fails the zero
    location pin and, for p = 4, the published table."""
    alt = _reflected_pair_taps(p)
    k = db.tap_indices(p).astype(float)
    assert abs(alt.sum() - 1) < 1e-13
    for j in range(p):
        assert abs(np.sum((-1) ** k * (k / p) ** j * alt)) < 1e-12
    for l in range(1, p):
        assert abs(np.dot(alt[:-2 * l], alt[2 * l:])) < 1e-12
    assert abs(np.dot(alt, alt) - 0.5) < 1e-12
    assert np.max(np.abs(alt - db.filter_taps(p))) > 1e-3
    assert np.min(np.abs(_zeros_off_minus_one(alt, p))) < 1.0
    if p == 4:
        want = np.array(_golden("db4_taps.txt")["h_sqrt2"]) / math.sqrt(2.0)
        assert np.max(np.abs(alt - want)) > 1e-3


# ---------------------------------------------------------------- phi-hat (O2)

def test_haar_product_matches_closed_form():
    """P1: App. A prints F[phi] for Haar in closed form, 1 at 0."""
    xi = np.concatenate([np.linspace(-40, 40, 801), [0.0, 1e-9, -3.0, 7.5]])
    got = db.phi_hat(xi, 1)
    import mpmath
    with mpmath.workdps(40):
        want = np.array([complex((1 - mpmath.expj(-2 * mpmath.pi * mpmath.mpf(float(x))))
                                 / (2j * mpmath.pi * mpmath.mpf(float(x)))) if x != 0 else 1.0
                         for x in xi])
    assert np.max(np.abs(got - want)) < 2e-15
    assert db.phi_hat(np.array([0.0]), 1)[0] == 1.0


def test_product_start_index():
    """The product must start at j = 1: starting at j = 0 multiplies by m0(xi)
    and breaks the Haar closed form."""
    xi = np.array([0.37, 1.3, -2.6])
    wrong = db.m0(xi, 1) * db.phi_hat(xi, 1)
    assert np.max(np.abs(wrong - db.haar_phi_hat_closed_form(xi))) > 0.1


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_phi_hat_invariants(p):
    """P2: phi-hat(0) = 1, zeros at the nonzero integers, Hermitian symmetry,
    and the orthonormality identity sum_k |phi-hat(eta + k)|^2 = 1."""
    assert abs(db.phi_hat(np.array([0.0]), p)[0] - 1) < 1e-15
    ints = np.array([-5.0, -2.0, -1.0, 1.0, 3.0, 8.0])
    assert np.max(np.abs(db.phi_hat(ints, p))) < 1e-14
    eta = np.array([0.1, 0.37, 1.9, -4.2])
    assert np.max(np.abs(db.phi_hat(-eta, p) - np.conj(db.phi_hat(eta, p)))) < 1e-15
    # partial sums over |k| <= K increase to exactly 1: the missing tail is
    # non-negative and shrinks as K grows
    tol = {2: 1e-7, 3: 1e-10, 4: 1e-12, 6: 1e-13}[p]
    for e in [0.13, 0.5, 0.81]:
        tails = []
        for K in (1000, 4000):
            s = np.sum(np.abs(db.phi_hat(e + np.arange(-K, K + 1, dtype=float), p)) ** 2)
            tails.append(1 - s)
        assert tails[0] > -1e-13 and tails[1] > -1e-13
        assert tails[1] <= tails[0] + 1e-14
        assert tails[1] < tol


@pytest.mark.parametrize("p", [2, 3, 4])
def test_phi_hat_against_space_domain(p):
    """Independent route: phi on a dyadic grid from the refinement equation
    (cascade), Fourier transform by quadrature."""
    x, ph = cascade.phi_on_grid(p, 13)
    xi = np.array([0.0, 0.3, 1.7, -2.2, 3.9])
    err = np.max(np.abs(cascade.trapezoid_ft(x, ph, xi) - db.phi_hat(xi, p)))
    assert err < 1e-7


# ------------------------------------------------- boundary functions (O3)

@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("side", ["left", "right"])
def test_boundary_filter_structure(p, side):
    """P3: V has the staircase printed in App. A.1 (row k non-zero only for
    m = p..p+2k); eig(U) = {2^-1 .. 2^-p} (the boundary functions reproduce
    polynomials of degree < p near the edge); each row of [H h] has unit norm
    (the dilation equation is an orthonormal expansion)."""
    e = cdv.left_edge(p) if side == "left" else cdv.flipped_edge(p)
    U, V = e.U(), e.V()
    assert float(e.gram_residual) < 1e-40
    for k in range(p):
        nz = np.nonzero(np.abs(V[k]) > 1e-15)[0]
        assert nz.max() <= 2 * k, (k, nz)
        assert abs(V[k, 2 * k]) > 1e-6
    ev = np.sort(np.linalg.eigvals(U).real)[::-1]
    assert np.allclose(ev, 2.0 ** -np.arange(1, p + 1), atol=1e-12)
    assert np.allclose(2 * (U ** 2).sum(1) + 2 * (V ** 2).sum(1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_v1_zero_two_routes(p):
    """P4: the xi = 0 system of App. A.1 solved by QR equals the integrals of
    the boundary functions computed from their translate coefficients and the
    partition of unity."""
    for e in (cdv.left_edge(p), cdv.flipped_edge(p)):
        v = e.v1_zero()
        assert np.max(np.abs(v - e.integrals())) < 1e-14
        U, V = e.U(), e.V()
        assert np.max(np.abs(v - U @ v - V @ np.ones(2 * p - 1))) < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4])
def test_boundary_functions_against_space_domain(p):
    """Independent route for the whole boundary construction: build phi^L_k and
    phi^R_k in space from the cascade values of phi, check orthonormality and
    orthogonality to the interior translates by quadrature, and compare their
    numerical Fourier transforms with the dilation recursion."""
    R = 13
    x, ph = cascade.phi_on_grid(p, R)
    xi = np.array([0.0, 0.45, -1.3, 2.75])
    for side in ("left", "right"):
        e = cdv.left_edge(p) if side == "left" else cdv.flipped_edge(p)
        A = e.coef_fp64()
        if side == "left":
            xs = np.arange(0, 2 * p * 2 ** R + 1) / 2 ** R
            f = np.array([sum(A[k, i] * cascade.eval_translates(x, ph, R, xs, n)
                              for i, n in enumerate(e.trans)) for k in range(p)])
            interior = [cascade.eval_translates(x, ph, R, xs, n) for n in range(p, 2 * p + 1)]
            want = cdv.left_phi_hat(xi, p)
        else:
            xs = -(np.arange(0, 2 * p * 2 ** R + 1) / 2 ** R)[::-1]
            f = np.array([sum(A[k, i] * cascade.eval_translates(x, ph, R, 1 + xs + n, 0)
                              for i, n in enumerate(e.trans)) for k in range(p)])
            interior = [cascade.eval_translates(x, ph, R, xs, -n - 1) for n in range(p, 2 * p + 1)]
            want = cdv.right_phi_hat(xi, p)
        G = np.array([[cascade.trapezoid_inner(xs, f[a], f[b]) for b in range(p)] for a in range(p)])
        assert np.max(np.abs(G - np.eye(p))) < 1e-6
        cross = [cascade.trapezoid_inner(xs, f[a], g) for a in range(p) for g in interior]
        assert np.max(np.abs(cross)) < 1e-6
        F = np.array([cascade.trapezoid_ft(xs, f[k], xi) for k in range(p)])
        assert np.max(np.abs(F - want)) < 1e-6


# ------------------------------------------------------------ basis T (O4)

@pytest.mark.parametrize("p,J", [(1, 4), (2, 3), (2, 5), (3, 4), (4, 4), (4, 6), (2, 2), (4, 3)])
def test_sinc_identity(p, J):
    """P9: 1_[-1/2,1/2] lies in V_J^int and the basis is orthonormal, so
    sum_n b_n(0) b_n(xi) = sin(pi xi)/(pi xi) for every xi and
    sum_n b_n(0)^2 = 1.  Exercises interior phases, boundary phases and the
    boundary functions together."""
    b0 = basis.columns_1d(np.array([0.0]), J, p)[:, 0]
    assert np.max(np.abs(b0.imag)) < 1e-15
    assert abs(np.sum(b0.real ** 2) - 1) < 1e-13
    xs = np.concatenate([np.linspace(-70, 70, 141) + 0.31, [0.5, -0.5, 17.0]])
    got = b0 @ basis.columns_1d(xs, J, p)
    assert np.max(np.abs(got - np.sinc(xs))) < 5e-14


@pytest.mark.parametrize("p,J", [(1, 3), (2, 3), (4, 4), (3, 5)])
def test_gram_under_dense_uniform_sampling(p, J):
    """P8: with xi on the integers and mu = 1 the samples are Fourier series
    coefficients on an interval of length 1, so T^H W T -> I as the band
    [-B, B] grows (Parseval).  The missing tail d_n = 1 - G_nn is
    non-negative, shrinks like 1/B, and bounds every off-diagonal entry by
    Cauchy-Schwarz."""
    N = 1 << J
    Gs = []
    for B in (2000, 8000):
        xi = np.arange(-B, B + 1, dtype=float)
        T = basis.dense_T_1d(xi, J, p)
        Gs.append(T.conj().T @ T)
    for G, B in zip(Gs, (2000, 8000)):
        d = 1 - np.diag(G).real
        assert np.all(d > -1e-13)
        assert d.max() < 40.0 * N / B
        off = np.abs(G - np.diag(np.diag(G)))
        assert np.all(off <= np.sqrt(np.outer(d, d)) + 1e-12)
    d1 = 1 - np.diag(Gs[0]).real
    d2 = 1 - np.diag(Gs[1]).real
    assert np.all(d2 < 0.3 * d1 + 1e-13)
    # half-integer sampling with mu = 1/2 is also a tight frame
    xi = np.arange(-8000, 8000.5, 0.5)
    T = basis.dense_T_1d(xi, J, p)
    G = 0.5 * T.conj().T @ T
    d = 1 - np.diag(G).real
    assert d.max() < 40.0 * N / 8000


def test_haar_rows_are_scaled_ndft():
    """For Haar, T = D F with F the NDFT matrix of Sec. 3.2 at eta = 2^-J xi,
    checked against the independent NDFT code."""
    J, N = 4, 16
    rng = np.random.default_rng(0)
    xi = rng.uniform(-30, 30, 50)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    D = 2 ** (-J / 2) * db.haar_phi_hat_closed_form(xi / N)
    assert np.max(np.abs(basis.dense_T_1d(xi, J, 1) @ x - D * ndft.ndft_1d(x, xi / N))) < 1e-13


def test_2d_rows_are_kronecker_products():
    """P10 (App. C): one frequency, p = 2, six functions per dimension in the
    paper's example; here N = 8.  Row of the 2D matrix = outer product of 1D
    rows; the matrix-free product equals the dense one."""
    J, p = 3, 2
    rng = np.random.default_rng(1)
    xi2 = rng.uniform(-9, 9, (7, 2))
    T2 = basis.dense_T_2d(xi2, J, p)
    bx = basis.columns_1d(xi2[:, 0], J, p)
    by = basis.columns_1d(xi2[:, 1], J, p)
    for m in range(7):
        assert np.allclose(T2[m].reshape(8, 8), np.outer(bx[:, m], by[:, m]), atol=1e-15)
    X = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    assert np.max(np.abs(basis.apply_T_2d(xi2, J, p, X) - T2 @ X.reshape(-1))) < 1e-13
    u = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    assert np.max(np.abs(basis.apply_TH_2d(xi2, J, p, u).reshape(-1) - T2.conj().T @ u)) < 1e-13


def test_2d_haar_against_2d_ndft():
    J, N = 3, 8
    rng = np.random.default_rng(2)
    xi2 = rng.uniform(-20, 20, (30, 2))
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    D = (2 ** (-J / 2)) ** 2 * db.haar_phi_hat_closed_form(xi2[:, 0] / N) * db.haar_phi_hat_closed_form(xi2[:, 1] / N)
    want = D * ndft.ndft_2d(X, xi2 / N)
    assert np.max(np.abs(basis.apply_T_2d(xi2, J, 1, X) - want)) < 1e-13
    u = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    wantH = ndft.ndft_adjoint_2d(np.conj(D) * u, xi2 / N, N, N)
    assert np.max(np.abs(basis.apply_TH_2d(xi2, J, 1, u) - wantH)) < 1e-13


def test_selected_outputs_match_full_products():
    J, p = 4, 4
    rng = np.random.default_rng(3)
    xi2 = rng.uniform(-16, 16, (300, 2))
    X = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    u = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    y = basis.apply_T_2d(xi2, J, p, X)
    rows = np.array([0, 17, 299])
    assert np.allclose(basis.rows_T_2d(xi2, J, p, X, rows), y[rows], atol=1e-14)
    Z = basis.apply_TH_2d(xi2, J, p, u)
    ij = np.array([[0, 0], [3, 15], [15, 2], [7, 8]])
    assert np.allclose(basis.coeffs_TH_2d(xi2, J, p, u, ij), Z[ij[:, 0], ij[:, 1]], atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_single_column_matches_all_columns(p):
    J = 5
    xi = np.random.default_rng(4).uniform(-40, 40, 500)
    B = basis.columns_1d(xi, J, p)
    for n in (0, 1, p - 1, p, 16, 31 - p, 31 - p + 1, 31):
        assert np.array_equal(basis.column_1d(xi, J, p, n), B[n])
    ns = [0, p - 1, p, 16, 31 - p, 31]
    sub = basis.columns_subset_1d(xi, J, p, ns)
    assert sorted(sub) == sorted(set(ns))
    for n in ns:
        assert np.array_equal(sub[n], B[n])


# ------------------------------------------------------------------ NDFT (O5)

def test_ndft_uniform_reduces_to_dft():
    """P6 (Sec. 3.2): for xi_m = eps (m-1-M/2)/N, eps^-1 integer, the NDFT is
    the first M entries of the DFT of a zero-interleaved, phase-shifted vector
    (here computed with numpy.fft)."""
    N1, N, M, eps = 8, 16, 24, 0.5
    rng = np.random.default_rng(4)
    x = rng.standard_normal(N1) + 1j * rng.standard_normal(N1)
    m = np.arange(1, M + 1)
    xi = eps / N * (m - 1 - M / 2)
    q = 1
    while q * N / eps < M:
        q += 1
    N2 = int(q * N / eps)
    z = np.zeros(N2, complex)
    ell = np.arange(1, N1 + 1)
    z[q * (ell - 1)] = x * np.exp(1j * np.pi * (ell - 1) * eps * M / N)
    dft = np.fft.fft(z)[:M]
    want = np.exp(1j * np.pi * N1 * xi) * dft
    assert np.max(np.abs(ndft.ndft_1d(x, xi) - want)) < 1e-13


def test_ndft_against_mpmath_and_adjoint():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    xi = rng.uniform(-0.5, 0.5, 5)
    assert np.max(np.abs(ndft.ndft_1d(x, xi) - ndft.ndft_1d_mp(x, xi))) < 1e-14
    y = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    lhs = np.vdot(y, ndft.ndft_1d(x, xi))
    rhs = np.vdot(ndft.ndft_adjoint_1d(y, xi, 6), x)
    assert abs(lhs - rhs) < 1e-13


# ------------------------------------------------------------ LS (O6, O7)

@pytest.mark.parametrize("p", [1, 2, 4])
def test_cgls_matches_lstsq(p):
    """P11: CGLS reaches the library least-squares solution; the normal
    equations hold."""
    J = 5
    rng = np.random.default_rng(6)
    xi = np.sort(rng.uniform(-64, 64, 200))
    mu = np.gradient(xi)
    T = basis.dense_T_1d(xi, J, p)
    y = T @ (rng.standard_normal(32) + 0j) + 1e-3 * rng.standard_normal(200)
    x_ref = lsq.lstsq_dense(T, y, mu)
    s = np.sqrt(mu)
    A = T * s[:, None]
    b = y * s
    x, it, hist = lsq.cgls(lambda v: A @ v, lambda v: A.conj().T @ v, b, np.zeros(32, complex), 1e-13, 500)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-10
    assert lsq.normal_residual(lambda v: A @ v, lambda v: A.conj().T @ v, b, x) < 1e-12
    assert hist[-1] <= 1e-13 and it < 200
