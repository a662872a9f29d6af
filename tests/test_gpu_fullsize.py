"""Full-size parity at the benchmark shape: 2D db4 at J = 9 (512 x 512
coefficients), 1,048,576 Archimedean-spiral points (64 arms x 16384, radius
256), mixed-precision plan, weighted operator, caller point order -- the
launch configuration the benchmark times -- and at the warm-start workload's
shape (J = 8, 256 x 256, 64 arms x 4096 points, radius 128).  The FP64
oracle cannot form the full products at these sizes, so:

  * T x is compared on 128 sampled outputs, each row formed by the oracle;
  * T^H u is compared on 12 coefficients (boundary and interior indices) for
    an input u that is nonzero on 20,000 seeded points spread over the whole
    plane and zero elsewhere: the GPU still runs the full launch over every
    tile, while the oracle's coefficient sums need only the support;
  * the adjoint identity <T x, u> = <x, T^H u> is checked with a dense u.

Tolerances: relative error <= 1e-12 (FP64 applies), <= 2e-5 (FP32 applies),
over the sampled vectors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis
from workloads import spiral_2d

from gpu_util import rel, crandn, to_dev, to_host, say

pytestmark = pytest.mark.gpu

P = 4
SHAPES = {"spiral_1M_J9": (9, 16384, 256.0), "spiral_262k_J8": (8, 4096, 128.0)}


@pytest.fixture(scope="module", params=list(SHAPES))
def setup(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs
    J, per_arm, r_max = SHAPES[request.param]
    pts = spiral_2d(64, per_arm, r_max, 0.5)
    rng = np.random.default_rng(2024)
    mu = rng.uniform(0.5, 1.5, pts.shape[0])
    plan = gs.gs_plan(2, J, P, pts, mu, precision=gs.GS_F32_MIXED)
    yield gs, plan, pts, mu, J
    plan.destroy()


def _dtype(f64):
    return torch.complex128 if f64 else torch.complex64


@pytest.mark.parametrize("f64", [True, False])
def test_forward_sampled_rows(setup, f64):
    gs, plan, pts, mu, J = setup
    N = 1 << J
    say(f"[fullsize T] M={pts.shape[0]} f64={f64}")
    rng = np.random.default_rng(11)
    X = crandn(rng, (N, N))
    y = to_host(plan.apply_T(to_dev(X, _dtype(f64)), weighted=True, f64=f64))
    rows = np.sort(rng.choice(pts.shape[0], 128, replace=False))
    want = np.sqrt(mu[rows]) * basis.rows_T_2d(pts, J, P, X, rows)
    assert rel(y[rows], want) < (1e-12 if f64 else 2e-5)


@pytest.mark.parametrize("f64", [True, False])
def test_adjoint_sampled_coefficients(setup, f64):
    gs, plan, pts, mu, J = setup
    N = 1 << J
    say(f"[fullsize T^H] M={pts.shape[0]} f64={f64}")
    rng = np.random.default_rng(12)
    M = pts.shape[0]
    support = np.sort(rng.choice(M, 20000, replace=False))
    u = np.zeros(M, dtype=np.complex128)
    u[support] = crandn(rng, support.size)
    Z = to_host(plan.apply_TH(to_dev(u, _dtype(f64)), weighted=True, f64=f64))
    ij = np.array([[0, 0], [0, N - 1], [3, 4], [4, N // 2 - 1], [N // 2, N // 2 + 1], [N - 4, 3],
                   [N - 1, N - 1], [N // 5, 4 * N // 5], [N // 2, 7], [2, 3 * N // 5], [N - 3, N - 2],
                   [N // 4, N // 4 + 1]])
    want = basis.coeffs_TH_2d(pts[support], J, P, np.sqrt(mu[support]) * u[support], ij)
    assert rel(Z[ij[:, 0], ij[:, 1]], want) < (1e-12 if f64 else 2e-5)


@pytest.mark.parametrize("f64", [True, False])
def test_adjoint_identity_dense(setup, f64):
    gs, plan, pts, mu, J = setup
    N = 1 << J
    say(f"[fullsize adjoint identity] f64={f64}")
    rng = np.random.default_rng(13)
    X = crandn(rng, (N, N))
    u = crandn(rng, pts.shape[0])
    dt = _dtype(f64)
    y = to_host(plan.apply_T(to_dev(X, dt), weighted=True, f64=f64))
    Z = to_host(plan.apply_TH(to_dev(u, dt), weighted=True, f64=f64))
    lhs = np.vdot(u, y)
    rhs = np.vdot(Z, X)
    scale = np.linalg.norm(u) * np.linalg.norm(y)
    assert abs(lhs - rhs) / scale < (1e-13 if f64 else 1e-6)
