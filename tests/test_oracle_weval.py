"""Pins of the oracle's evaluation in space (oracle.cascade.weval, the weval
of Sec. 6.2) against what the paper and the mathematics fix:

* Haar: the closed form f(x) = 2^{J/2} x_n on [n/N - 1/2, (n+1)/N - 1/2);
* the constant 1 on [-1/2, 1/2] lies in V_J^int, and its coefficients are
  <s_n, 1> = s_n-hat(0) = b_n(0), the Fourier-side columns at xi = 0 (Sec. 4):
  weval of b(0) must be 1 at every grid point -- the space construction
  (cascade, restricted translates) against the Fourier construction (infinite
  product, dilation recursion), two routes that share no step;
* linear functions (p >= 2): <s_n, x> = i/(2 pi) d/dxi b_n(xi) at 0 (central
  differences of the Fourier-side columns), and weval returns x;
* orthonormality: the trapezoid integral of |f|^2 equals sum |x_n|^2;
* 2D: the tensor product of the 1D evaluations."""
import numpy as np
import pytest

from oracle import basis, cascade


@pytest.mark.parametrize("J,R", [(3, 6), (5, 10)])
def test_haar_closed_form(J, R):
    rng = np.random.default_rng(J)
    N = 1 << J
    c = rng.standard_normal(N)
    x, f = cascade.weval(c, J, 1, R)
    n = np.floor((x + 0.5) * N).astype(int)
    want = np.where(n < N, 2 ** (J / 2) * c[np.minimum(n, N - 1)], 0.0)
    assert np.max(np.abs(f - want)) < 1e-13


@pytest.mark.parametrize("p,J", [(2, 3), (2, 5), (3, 4), (4, 3), (4, 5), (5, 4)])
def test_constant_from_fourier_side_columns(p, J):
    b0 = basis.columns_1d(np.array([0.0]), J, p)[:, 0]
    assert np.max(np.abs(b0.imag)) < 1e-14
    x, f = cascade.weval(b0.real, J, p, J + 7)
    assert np.max(np.abs(f - 1.0)) < 1e-12


@pytest.mark.parametrize("p,J", [(2, 4), (3, 4), (4, 5)])
def test_linear_from_fourier_side_derivative(p, J):
    d = 1e-4
    bp = basis.columns_1d(np.array([d]), J, p)[:, 0]
    bm = basis.columns_1d(np.array([-d]), J, p)[:, 0]
    c = 1j / (2 * np.pi) * (bp - bm) / (2 * d)           # <s_n, x> = i/(2 pi) b_n'(0)
    assert np.max(np.abs(c.imag)) < 1e-9
    x, f = cascade.weval(c.real, J, p, J + 6)
    assert np.max(np.abs(f - x)) < 1e-7


@pytest.mark.parametrize("p,J", [(1, 4), (2, 4), (4, 4)])
def test_orthonormal_basis(p, J):
    rng = np.random.default_rng(7)
    N = 1 << J
    c = rng.standard_normal(N)
    x, f = cascade.weval(c, J, p, J + 10)
    h = x[1] - x[0]
    integral = h * (np.sum(f ** 2) - 0.5 * (f[0] ** 2 + f[-1] ** 2))
    assert abs(integral - np.sum(c ** 2)) / np.sum(c ** 2) < 2e-4


def test_2d_is_the_tensor_product():
    rng = np.random.default_rng(9)
    J, p, R = 3, 2, 6
    X = rng.standard_normal((8, 8))
    x, F = cascade.weval(X, J, p, R)
    _, S = cascade.basis_on_grid(J, p, R)
    a, b = 13, 50
    want = sum(X[i, j] * S[i, a] * S[j, b] for i in range(8) for j in range(8))
    assert abs(F[a, b] - want) < 1e-12
