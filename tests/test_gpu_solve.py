"""GPU CGLS (gs_solve) against the oracle's least-squares solution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis, lsq
from workloads import config_c1, complex_noise, spiral_2d, jitter_2d, voronoi_weights_2d, ellipse_phantom_params, \
    phantom_cell_averages

from gpu_util import assert_close, rel, crandn, to_dev, to_host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs as _gs
    return _gs


def test_c1_solve_matches_lstsq(gs):
    """1D db2, J=8, 1024 uniform points, noisy data: the GPU CGLS (FP64,
    solved to 1e-10) is within 1e-6 of the library least-squares solution."""
    say("[c1 solve]")
    c = config_c1()
    J, p, xi = c["J"], c["p"], c["xi"]
    T = basis.dense_T_1d(xi, J, p)
    y = T @ c["x0"] + complex_noise(xi.size, c["noise_sigma"], c["noise_seed"])
    x_ref = lsq.lstsq_dense(T, y)
    plan = gs.gs_plan(1, J, p, xi, None, precision=gs.GS_F64)
    x, info = plan.solve(to_dev(y, torch.complex128), rel_tol=c["tol"], max_iter=500, history=True)
    assert info["status"] == gs.GS_OK
    assert info["rel_residual"] <= c["tol"]
    assert_close(to_host(x), x_ref, 1e-6, "x")
    assert len(info["history"]) == info["iterations"] + 1
    # the same recurrence on the oracle's dense matrices
    _, it_ref, _ = lsq.cgls(lambda v: T @ v, lambda v: T.conj().T @ v, y, np.zeros(256, complex), c["tol"], 500)
    assert abs(info["iterations"] - it_ref) <= 2
    plan.destroy()


def _small_2d(J=5, p=4, pattern="spiral", seed=301):
    """Well-conditioned 2D test problems.  A spiral of radius N/2 (the shape of
    the 1M-point workload) leaves the corners of the coefficient band
    unsampled and is numerically rank deficient (condition number ~1e9 at
    J = 5), so least-squares parity uses a spiral of radius 0.75 N
    (condition ~2e2) and a jittered grid over [-N, N]^2 (condition ~3)."""
    N = 1 << J
    if pattern == "spiral":
        pts = spiral_2d(64, 140 * N // 32, 0.75 * N, 0.5)
        mu = voronoi_weights_2d(pts, "disk", 0.75 * N + 0.25, 0.4)
    else:
        pts = jitter_2d(4 * N * N, N, seed)
        mu = voronoi_weights_2d(pts, "square", N, 1.0)
    x0 = phantom_cell_averages(ellipse_phantom_params(seed), J).astype(complex)
    return pts, mu, x0


@pytest.mark.parametrize("pattern,prec", [("spiral", 0), ("jitter", 0), ("jitter", 2), ("spiral", 2)])
def test_2d_weighted_solve_matches_lstsq(gs, pattern, prec):
    """Plain FP64 and FP32-mixed solves to a normal residual of 1e-10 are
    within 1e-6 of the oracle's weighted LS solution, element by element.  The
    mixed form reaches 1e-10 through its FP64 refinement restarts (each one
    gains about the FP32 accuracy on the remaining error)."""
    say(f"[2d solve] {pattern} prec={prec}")
    J, p = 5, 4
    pts, mu, x0 = _small_2d(J, p, pattern)
    T = basis.dense_T_2d(pts, J, p)
    y = T @ x0.reshape(-1)
    y = y + complex_noise(y.size, 1e-4 * np.linalg.norm(y) / np.sqrt(2 * y.size), 302)
    x_ref = lsq.lstsq_dense(T, y, mu).reshape(32, 32)
    plan = gs.gs_plan(2, J, p, pts, mu, precision=prec)
    tol = 1e-10
    x, info = plan.solve(to_dev(y, torch.complex128), rel_tol=tol, max_iter=1000, refine_fp64=True,
                         max_restarts=8)
    say(f"  iters={info['iterations']} restarts={info['restarts']} rr={info['rel_residual']:.2e} "
        f"rr64={info['rel_residual_fp64']:.2e}")
    assert info["status"] == gs.GS_OK
    if prec == 2:
        assert info["rel_residual_fp64"] <= tol
    assert_close(to_host(x), x_ref, 1e-6, "x vs oracle LS")
    plan.destroy()


def test_f32_plan_below_its_floor(gs):
    """A plain FP32 plan asked for a tolerance below FP32 accuracy on
    inconsistent data: the recurrence stalls, which is a stop, not a
    breakdown.  The status is GS_NOT_CONVERGED and x is the run's best
    iterate: finite, with a small true (oracle) normal residual."""
    say("[f32 floor]")
    J, p = 5, 2
    pts, mu, _ = _small_2d(J, p, "jitter")
    y = crandn(np.random.default_rng(78), pts.shape[0])
    plan = gs.gs_plan(2, J, p, pts, mu, precision=gs.GS_F32)
    x, info = plan.solve(to_dev(y, torch.complex128), rel_tol=1e-12, max_iter=600)
    xh = to_host(x).reshape(-1)
    T = basis.dense_T_2d(pts, J, p)
    w = mu
    g0 = np.linalg.norm(T.conj().T @ (w * y))
    g = np.linalg.norm(T.conj().T @ (w * (y - T @ xh)))
    say(f"  status={info['status']} iters={info['iterations']} rr={info['rel_residual']:.2e} true={g / g0:.2e}")
    assert info["status"] == gs.GS_NOT_CONVERGED
    assert info["iterations"] < 600
    assert np.isfinite(xh).all()
    assert g / g0 < 1e-4
    plan.destroy()


def test_warm_start_and_limits(gs):
    say("[warm start / limits]")
    J, p = 5, 2
    pts, mu, x0 = _small_2d(J, p, "jitter", seed=77)
    T = basis.dense_T_2d(pts, J, p)
    y = T @ x0.reshape(-1)
    plan = gs.gs_plan(2, J, p, pts, mu, precision=0)
    yd = to_dev(y, torch.complex128)
    x_cold, info_cold = plan.solve(yd, rel_tol=1e-8, max_iter=300)
    xw = to_dev(x0 * (1 + 1e-3), torch.complex128).reshape(32, 32).contiguous()
    x_warm, info_warm = plan.solve(yd, xw, rel_tol=1e-8, max_iter=300, warm_start=True)
    assert info_warm["status"] == gs.GS_OK and info_cold["status"] == gs.GS_OK
    assert info_warm["iterations"] < info_cold["iterations"]
    assert_close(to_host(x_warm), to_host(x_cold), 1e-6, "x_warm")
    # max_iter reached -> positive status, x holds the last iterate
    x1, info1 = plan.solve(yd, rel_tol=1e-14, max_iter=1)
    assert info1["status"] == gs.GS_NOT_CONVERGED and info1["iterations"] == 1
    # y = 0 -> x = 0 immediately
    xz, infz = plan.solve(torch.zeros_like(yd), rel_tol=1e-8, max_iter=10)
    assert infz["status"] == gs.GS_OK and infz["iterations"] == 0
    assert float(torch.abs(xz).max()) == 0.0
    # check_every > 1 gives the same result as checking every iteration
    xa, ia = plan.solve(yd, rel_tol=1e-8, max_iter=300, check_every=7)
    assert ia["iterations"] == info_cold["iterations"]
    assert torch.equal(xa, x_cold)
    plan.destroy()


@pytest.mark.parametrize("J,p,pattern", [(4, 2, "jitter"), (5, 2, "spiral")])
def test_mixed_below_fp32_floor_is_graceful(gs, J, p, pattern):
    """An inconsistent problem (random data) asked for a tolerance below what
    FP32 applies can reach: the FP32 recurrence stalls, the FP64 residual is
    recomputed and the recurrence restarted; the result is GS_OK or
    GS_NOT_CONVERGED with a finite iterate whose FP64 normal residual is small,
    never a breakdown."""
    say(f"[mixed floor] J={J} p={p} {pattern}")
    N = 1 << J
    pts, mu, _ = _small_2d(J, p, pattern)
    y = crandn(np.random.default_rng(77), pts.shape[0])
    plan = gs.gs_plan(2, J, p, pts, mu, precision=gs.GS_F32_MIXED)
    x, info = plan.solve(to_dev(y, torch.complex128), rel_tol=1e-9, max_iter=400, refine_fp64=True,
                         max_restarts=3)
    xh = to_host(x)
    say(f"  status={info['status']} iters={info['iterations']} restarts={info['restarts']} "
        f"rr64={info['rel_residual_fp64']:.2e}")
    assert info["status"] in (gs.GS_OK, gs.GS_NOT_CONVERGED)
    assert np.isfinite(xh).all()
    assert 0 <= info["rel_residual_fp64"] < 1e-4
    # its weighted LS objective is that of the oracle's LS solution, to 1e-6
    T = basis.dense_T_2d(pts, J, p)
    x_ref = lsq.lstsq_dense(T, y, mu)
    w = np.sqrt(mu)

    def objective(v):
        return np.linalg.norm(w * (T @ v - y))

    assert objective(xh.reshape(-1)) <= objective(x_ref) * (1 + 1e-6)
    plan.destroy()


@pytest.mark.parametrize("prec", [0, 2])
def test_check_interval_does_not_change_the_result(gs, prec):
    """Where the host checks the stop flag (every iteration, every few, or at
    intervals the convergence rate shortens near the tolerance) changes only
    how many queued iterations run after the stop, and those leave every
    vector as it is: the solution and the iteration count are identical bit
    for bit whatever check_every is."""
    say(f"[check interval] prec={prec}")
    J, p = 5, 4
    pts, mu, x0 = _small_2d(J, p, "spiral")
    T = basis.dense_T_2d(pts, J, p)
    y = T @ x0.reshape(-1)
    y = y + complex_noise(y.size, 1e-4 * np.linalg.norm(y) / np.sqrt(2 * y.size), 303)
    plan = gs.gs_plan(2, J, p, pts, mu, precision=prec)
    yd = to_dev(y, torch.complex128)
    runs = []
    for ce in (1, 3, 10, 64):
        x, info = plan.solve(yd, rel_tol=1e-9, max_iter=400, refine_fp64=True, max_restarts=4, check_every=ce)
        say(f"  check_every={ce}: iters={info['iterations']} restarts={info['restarts']}")
        assert info["status"] == gs.GS_OK
        runs.append((x, info))
    x1, i1 = runs[0]
    for x, info in runs[1:]:
        assert info["iterations"] == i1["iterations"] and info["restarts"] == i1["restarts"]
        assert info["rel_residual"] == i1["rel_residual"]
        assert torch.equal(x, x1)
    plan.destroy()


@pytest.mark.parametrize("prec", [0, 2])
def test_grid_below_a_tile_solve_matches_lstsq(gs, prec):
    """2D at J = 3: the NFFT grid (16 x 16) is narrower than a tile, so the
    applies take the plain 2D path and the CGLS norms come from the separate
    reduction instead of the tile path's fused partial sums.  Plain FP64 and
    FP32-mixed solves to 1e-10 are within 1e-6 of the oracle's weighted LS
    solution, element by element, and independent of the check interval."""
    say(f"[grid below a tile] prec={prec}")
    J, p = 3, 2
    N = 1 << J
    pts, mu, x0 = _small_2d(J, p, "jitter")
    T = basis.dense_T_2d(pts, J, p)
    y = T @ x0.reshape(-1)
    y = y + complex_noise(y.size, 1e-4 * np.linalg.norm(y) / np.sqrt(2 * y.size), 304)
    x_ref = lsq.lstsq_dense(T, y, mu).reshape(N, N)
    plan = gs.gs_plan(2, J, p, pts, mu, precision=prec)
    assert plan.info()["grid_n"] < 32
    yd = to_dev(y, torch.complex128)
    x, info = plan.solve(yd, rel_tol=1e-10, max_iter=500, refine_fp64=True, max_restarts=8)
    say(f"  iters={info['iterations']} restarts={info['restarts']} rr64={info['rel_residual_fp64']:.2e}")
    assert info["status"] == gs.GS_OK
    assert_close(to_host(x), x_ref, 1e-6, "x vs oracle LS")
    x7, info7 = plan.solve(yd, rel_tol=1e-10, max_iter=500, refine_fp64=True, max_restarts=8, check_every=7)
    assert info7["iterations"] == info["iterations"] and torch.equal(x7, x)
    plan.destroy()
