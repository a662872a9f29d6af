"""The learned warm start end to end, at a small size (db4, J = 6, a 64-arm
spiral of radius 32 with Voronoi weights): training pairs made by the
library's own batched CGLS, training on the CNN kernels, and the guarded
warm-started solve.  Passing means: every solve (zero and warm start)
reaches the tolerance -- the final residual is what counts -- and the warm
start needs fewer CGLS iterations on held-out phantoms.  A network whose
x0 is worse than x0 = 0 must be rejected, leaving exactly the zero-start
solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import spiral_2d, voronoi_weights_2d

from gpu_util import to_host, say

pytestmark = pytest.mark.gpu

J, P = 6, 4


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs, warmstart
    pts = spiral_2d(64, 256, 32.0, 0.5)
    mu = voronoi_weights_2d(pts, "disk", 32.25, 0.4)
    plans = [gs.gs_plan(2, J, P, pts, mu, precision=gs.GS_F32_MIXED) for _ in range(4)]
    yield gs, warmstart, plans
    for pl in plans:
        pl.destroy()


def test_warm_start_gain(setup):
    gs, ws, plans = setup
    say("[warm start] generating 512 training pairs")
    inputs, targets, iters = ws.generate(plans, np.arange(50000, 50512), J)
    say(f"  mean target iterations {np.mean(iters):.1f}")
    net = gs.Cnn(1 << J, 1 << J, 16)
    net.set_weights(gs.cnn_he_init(7, last_scale=0.1))
    net.input_scale = ws.fit_input_scale(inputs, targets)
    hist = ws.train(net, inputs, targets, epochs=8, batch=16, lr_max=2e-3, log_every=64)
    say(f"  loss {hist[0][1]:.3e} -> {hist[-1][1]:.3e}")
    assert hist[-1][1] < hist[0][1]
    rows = ws.evaluate(plans[0], net, np.arange(70000, 70008), J)
    s = ws.summarize(rows)
    say(f"  {s}")
    assert s["all_converged"]
    assert s["max_rr64_warm"] <= 1e-6 and s["max_rr64_zero"] <= 1e-6
    assert s["warm_iters_mean"] < s["zero_iters_mean"]
    net.destroy()


def test_guarded_warm_start_falls_back(setup):
    gs, ws, plans = setup
    say("[warm start] guarded fallback")
    plan = plans[1]
    net = gs.Cnn(1 << J, 1 << J, 1)
    net.set_weights(gs.cnn_he_init(8, last_scale=0.1))
    net.input_scale = 1e6          # x0 = 1e6 A^H b: far worse than x0 = 0
    from workloads import ellipse_phantom_params, phantom_cell_averages_torch
    x0 = phantom_cell_averages_torch([ellipse_phantom_params(70010)], J, "cuda")[0]
    y = ws._noisy_data(plan, x0, 1e-4, 123)
    xw, iw = ws.warm_solve(plan, y, net)
    xz, iz = plan.solve(y, rel_tol=1e-6, max_iter=1000, refine_fp64=True, max_restarts=3, check_every=10)
    assert not iw["warm_start_used"]
    assert iw["iterations"] == iz["iterations"] and iw["status"] == gs.GS_OK
    assert np.array_equal(to_host(xw), to_host(xz))
    net.destroy()


def test_shipped_weights_on_held_out_phantoms():
    """The committed network (paper_1607_04091_amd/weights/c5_cnn.npz, trained
    on the 262,144-point J = 8 workload) on 8 held-out phantoms (seeds
    70000..70007) of that workload: every solve, warm and zero start, ends at
    an FP64 normal residual <= 1e-6, every warm start is kept by the guard,
    and the warm start needs fewer CGLS iterations on average (the bench
    measures -31 % on 100 phantoms)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import os
    from paper_1607_04091_amd import gs, warmstart as ws
    path = os.path.join(os.path.dirname(ws.__file__), "weights", "c5_cnn.npz")
    assert os.path.exists(path)
    say("[warm start] shipped weights, 8 held-out phantoms")
    plans, c = ws.c5_plans(1)
    N = 1 << c["J"]
    net = gs.Cnn(N, N, 1)
    net.load(path)
    rows = ws.evaluate(plans[0], net, np.arange(70000, 70008), c["J"])
    s = ws.summarize(rows)
    say(f"  {s}")
    assert s["all_converged"]
    assert s["max_rr64_warm"] <= 1e-6 and s["max_rr64_zero"] <= 1e-6
    assert s["warm_used"] == 8
    assert s["warm_iters_mean"] < 0.85 * s["zero_iters_mean"]
    net.destroy()
    plans[0].destroy()
