"""The size limits the library accepts, and the smallest cases.

* 2D at J = 11 (2048 x 2048 coefficients, a 4096^2 grid, 16,384 tiles) with
  100,000 random points over [-N, N]^2 (FP64 and FP32), and 1D at J = 20
  (2^20 coefficients, a 2^21-point grid on the four-step path) with 1,000,000
  random points (FP64: FP32 plans stop at J = 14, where a 32-bit position
  still has 17 bits of in-cell offset; 1D J = 14 in FP32 is the 65,536-point
  workload's size, tested at full size elsewhere): T x on sampled rows, and
  T^H u for a DENSE random u over all points on 32-34 sampled coefficients,
  against values the oracle summed over every point
  (tests/golden/make_dense_golden.py; inputs in tests/dense_cases.py);
* the smallest grids: Haar at J = 1 (N = 2) in 1D and 2D, and the largest
  wavelet order p = 8 (at J = 4, where 2^J = 2p: no interior columns; and at
  J = 5), against the dense oracle.
Tolerances: 1e-12 (FP64 applies), 2e-5 (FP32 applies), norm-wise and for the
worst element, with no exception for the smallest grids (the NFFT grid is never
narrower than the window)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis

import dense_cases

from gpu_util import assert_close, crandn, rel, to_dev, to_host, say

pytestmark = pytest.mark.gpu

TOL = {True: 1e-12, False: 2e-5}


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs as _gs
    return _gs


def _dt(f64):
    return torch.complex128 if f64 else torch.complex64


@pytest.mark.parametrize("f64", [True, False])
def test_2d_largest_grid(gs, f64):
    c = dense_cases.case("limits_2d_J11")
    J, p, pts = c["J"], c["p"], c["xi"]
    M, N = pts.shape[0], 1 << J
    say(f"[limits 2D] J={J} M={M} f64={f64}")
    rng = np.random.default_rng(111)
    plan = gs.gs_plan(2, J, p, pts, None, precision=gs.GS_F32_MIXED)
    X = crandn(rng, (N, N))
    y = to_host(plan.apply_T(to_dev(X, _dt(f64)), f64=f64))
    rows = np.sort(rng.choice(M, 48, replace=False))
    assert_close(y[rows], basis.rows_T_2d(pts, J, p, X, rows), TOL[f64], "T x rows")
    Z = to_host(plan.apply_TH(to_dev(c["u"], _dt(f64)), f64=f64))
    ij = c["idx"]
    assert_close(Z[ij[:, 0], ij[:, 1]], dense_cases.load_expected("limits_2d_J11"), TOL[f64], "T^H u samples")
    plan.destroy()


def test_1d_largest_grid(gs):
    c = dense_cases.case("limits_1d_J20")
    J, p, xi = c["J"], c["p"], c["xi"]
    M, N = xi.size, 1 << J
    f64 = True
    say(f"[limits 1D] J={J} M={M}")
    rng = np.random.default_rng(112)
    plan = gs.gs_plan(1, J, p, xi, None, precision=gs.GS_F64)
    x = crandn(rng, N)
    y = to_host(plan.apply_T(to_dev(x, _dt(f64)), f64=f64))
    rows = np.sort(rng.choice(M, 12, replace=False))
    assert_close(y[rows], basis.columns_1d(xi[rows], J, p).T @ x, TOL[f64], "T x rows")
    z = to_host(plan.apply_TH(to_dev(c["u"], _dt(f64)), f64=f64))
    assert_close(z[c["idx"]], dense_cases.load_expected("limits_1d_J20"), TOL[f64], "T^H u samples")
    plan.destroy()


@pytest.mark.parametrize("dim,J,p,M", [(1, 1, 1, 40), (2, 1, 1, 60), (1, 4, 8, 300), (2, 4, 8, 500),
                                       (2, 5, 8, 900)])
@pytest.mark.parametrize("prec", [0, 1])
def test_smallest_grids_and_largest_order(gs, dim, J, p, M, prec):
    say(f"[limits small] dim={dim} J={J} p={p} prec={prec}")
    rng = np.random.default_rng(113 + J + p + dim)
    N = 1 << J
    xi = rng.uniform(-1.5 * N, 1.5 * N, (M, 2) if dim == 2 else M)
    plan = gs.gs_plan(dim, J, p, xi, None, precision=prec)
    f64 = prec == 0
    shape = (N, N) if dim == 2 else (N,)
    x = crandn(rng, shape)
    u = crandn(rng, M)
    y = to_host(plan.apply_T(to_dev(x, _dt(f64))))
    z = to_host(plan.apply_TH(to_dev(u, _dt(f64))))
    T = basis.dense_T_2d(xi, J, p) if dim == 2 else basis.dense_T_1d(xi, J, p)
    assert_close(y, T @ x.reshape(-1), TOL[f64], "T x")
    assert_close(z.reshape(-1), T.conj().T @ u, TOL[f64], "T^H u")
    plan.destroy()
