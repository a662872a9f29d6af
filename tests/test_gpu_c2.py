"""The 1D nonuniform workload at full size: db4, J = 14 (16,384
coefficients), 65,536 jittered frequencies xi_k = (k + U(-1/4, 1/4)) / 2 with
Voronoi lengths, x0_i ~ N(0,1) / (1 + |i - 8192| / 512).  The dense oracle
T would be 65,536 x 16,384, so:

  * T x is compared on 128 sampled rows (the oracle forms each row);
  * T^H u on 34 sampled coefficients (edges and interior) for a DENSE random
    u over all points, against values the oracle summed over every point
    (tests/golden/make_dense_golden.py; inputs in tests/dense_cases.py);
  * the solves (FP64 plan; FP32-mixed plan) must recover x0 from the
    consistent data y = T x0 formed by the ORACLE (tests/golden/c2_y_oracle.npy,
    written by the same script): the jittered samples cover the whole band,
    so T has full column rank and the LS solution is x0.

Tolerances: 1e-12 (FP64 applies), 2e-5 (FP32 applies), norm-wise and for the
worst element; solves to a normal residual of 1e-8, x within 1e-6 of x0 (FP64)
and 1e-5 (mixed)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis
from workloads import config_c2

import dense_cases

from gpu_util import assert_close, crandn, rel, to_dev, to_host, say

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
    assert_close(y[rows], want, (1e-12 if f64 else 2e-5), "y")


@pytest.mark.parametrize("f64", [True, False])
def test_c2_adjoint_dense_sampled_coefficients(setup, f64):
    gs, plan, c = setup
    say(f"[c2 T^H dense] f64={f64}")
    d = dense_cases.case("c2_J14")
    dt = torch.complex128 if f64 else torch.complex64
    z = to_host(plan.apply_TH(to_dev(d["u"], dt), weighted=True, f64=f64))
    assert_close(z[d["idx"]], dense_cases.load_expected("c2_J14"), (1e-12 if f64 else 2e-5), "T^H u samples")


def _oracle_y():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_y_oracle.npy")
    return np.load(path, allow_pickle=False)


def test_c2_oracle_data_matches_fp64_apply(setup):
    """The stored oracle data y = T x0 against the library's FP64 apply, over
    all 65,536 rows."""
    gs, plan, c = setup
    say("[c2 oracle y]")
    y = to_host(plan.apply_T(to_dev(c["x0"], torch.complex128), f64=True))
    assert_close(y, _oracle_y(), 1e-12, "T x0 vs stored oracle y")


@pytest.mark.parametrize("prec", [0, 2])
def test_c2_solve_recovers_x0(setup, prec):
    gs, plan, c = setup
    say(f"[c2 solve] precision={prec}")
    x0 = c["x0"]
    y = to_dev(_oracle_y(), torch.complex128)
    pl = plan if prec == 2 else gs.gs_plan(1, J, P, c["xi"], c["mu"], precision=prec)
    x, info = pl.solve(y, rel_tol=1e-8, max_iter=500, refine_fp64=True, max_restarts=3, check_every=5)
    say(f"  status={info['status']} iters={info['iterations']} restarts={info['restarts']} "
        f"rr={info['rel_residual']:.2e} rr64={info['rel_residual_fp64']:.2e}")
    assert info["status"] == gs.GS_OK
    assert_close(to_host(x), x0, (1e-6 if prec == 0 else 1e-5), "x vs x0")
    if pl is not plan:
        pl.destroy()
