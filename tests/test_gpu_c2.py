"""The 1D nonuniform workload at full size: db4, J = 14 (16,384
coefficients), 65,536 jittered frequencies xi_k = (k + U(-1/4, 1/4)) / 2 with
Voronoi lengths, x0_i ~ N(0,1) / (1 + |i - 8192| / 512).  The dense oracle
T would be 65,536 x 16,384, so:

  * T x is compared on 128 sampled rows (the oracle forms each row);
  * T^H u on 16 coefficients (edges and interior) for u supported on 4,000
    seeded points;
  * the solves (FP64 plan; FP32-mixed plan) must recover x0 from the
    consistent data y = T x0: the jittered samples cover the whole band, so
    T has full column rank and the LS solution is x0.  y is made by the FP64
    apply, whose rows are checked against the oracle above.

Tolerances: 1e-12 (FP64 applies), 2e-5 (FP32 applies); solves to a normal
residual of 1e-8, x within 1e-6 of x0 (FP64) and 1e-5 (mixed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis
from workloads import config_c2

from gpu_util import crandn, rel, to_dev, to_host, say

pytestmark = pytest.mark.gpu

J, P = 14, 4
N = 1 << J


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs
    c = config_c2()
    plan = gs.gs_plan(1, J, P, c["xi"], c["mu"], precision=gs.GS_F32_MIXED)
    yield gs, plan, c
    plan.destroy()


@pytest.mark.parametrize("f64", [True, False])
def test_c2_forward_sampled_rows(setup, f64):
    gs, plan, c = setup
    say(f"[c2 T] f64={f64}")
    xi, mu, x0 = c["xi"], c["mu"], c["x0"]
    dt = torch.complex128 if f64 else torch.complex64
    y = to_host(plan.apply_T(to_dev(x0, dt), weighted=True, f64=f64))
    rows = np.sort(np.random.default_rng(21).choice(xi.size, 128, replace=False))
    want = np.sqrt(mu[rows]) * (basis.dense_T_1d(xi[rows], J, P) @ x0)
    assert rel(y[rows], want) < (1e-12 if f64 else 2e-5)


@pytest.mark.parametrize("f64", [True, False])
def test_c2_adjoint_sampled_coefficients(setup, f64):
    gs, plan, c = setup
    say(f"[c2 T^H] f64={f64}")
    xi, mu = c["xi"], c["mu"]
    rng = np.random.default_rng(22)
    support = np.sort(rng.choice(xi.size, 4000, replace=False))
    u = np.zeros(xi.size, dtype=np.complex128)
    u[support] = crandn(rng, support.size)
    dt = torch.complex128 if f64 else torch.complex64
    z = to_host(plan.apply_TH(to_dev(u, dt), weighted=True, f64=f64))
    idx = [0, 1, 3, 4, 100, N // 2 - 1, N // 2, 9000, N - 5, N - 4, N - 2, N - 1, 5, 8191, 12345, 2]
    wu = np.sqrt(mu[support]) * u[support]
    want = np.array([np.vdot(basis.column_1d(xi[support], J, P, n), wu) for n in idx])
    assert rel(z[idx], want) < (1e-12 if f64 else 2e-5)


@pytest.mark.parametrize("prec", [0, 2])
def test_c2_solve_recovers_x0(setup, prec):
    gs, plan, c = setup
    say(f"[c2 solve] precision={prec}")
    x0 = c["x0"]
    y = plan.apply_T(to_dev(x0, torch.complex128), f64=True)
    pl = plan if prec == 2 else gs.gs_plan(1, J, P, c["xi"], c["mu"], precision=prec)
    x, info = pl.solve(y, rel_tol=1e-8, max_iter=500, refine_fp64=True, max_restarts=3, check_every=5)
    err = rel(to_host(x), x0)
    say(f"  status={info['status']} iters={info['iterations']} restarts={info['restarts']} "
        f"rr={info['rel_residual']:.2e} rr64={info['rel_residual_fp64']:.2e} |x-x0|/|x0|={err:.2e}")
    assert info["status"] == gs.GS_OK
    assert err < (1e-6 if prec == 0 else 1e-5)
    if pl is not plan:
        pl.destroy()
