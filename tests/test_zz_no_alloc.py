"""The allocation-free adjoint entry point gs_apply_TH_noalloc, called through
the C ABI, against gs_apply_TH on the same plan and input: the results must
be bitwise equal (the same kernels in the same order, only the workspace
differs).  Two calls in a row share the static workspace, the second with a
smaller problem; a plan whose workspace exceeds the array is refused with
GS_ERR_TOO_LARGE before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import spiral_2d

from gpu_util import crandn, to_dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs as _gs
    return _gs


def _noalloc(gs, plan, u, x, flags):
    return gs.library().gs_apply_TH_noalloc(plan.handle, ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(x.data_ptr()), flags, None)


def _check(gs, plan, u, flags, dt):
    ref = torch.empty(plan.coef_shape(), dtype=dt, device="cuda")
    rc = gs.library().gs_apply_TH(plan.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                                  flags, None)
    assert rc == gs.GS_OK
    got = torch.full(plan.coef_shape(), complex(np.nan, np.nan), dtype=dt, device="cuda")
    rc = _noalloc(gs, plan, u, got, flags)
    assert rc == gs.GS_OK, gs.strerror(rc)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_equals_apply_TH_two_calls(gs):
    # call 1: 2D db4, J = 8, 262,144 spiral points, FP32 and FP64 (the larger workspace)
    pts = spiral_2d(64, 4096, 128.0, 0.5)
    mu = np.random.default_rng(5).uniform(0.5, 1.5, pts.shape[0])
    big = gs.gs_plan(2, 8, 4, pts, mu, precision=gs.GS_F32_MIXED)
    u = crandn(np.random.default_rng(6), pts.shape[0])
    for f64 in (False, True):
        dt = torch.complex128 if f64 else torch.complex64
        flags = gs.GS_WEIGHTED | (gs.GS_APPLY_F64 if f64 else 0)
        say(f"[noalloc] 2D J=8 M={pts.shape[0]} f64={f64}")
        _check(gs, big, to_dev(u, dt), flags, dt)
    # call 2: a smaller 2D problem (J = 5), then a 1D one, on the same array
    rng = np.random.default_rng(7)
    small = gs.gs_plan(2, 5, 2, rng.uniform(-20, 20, (3000, 2)), None, precision=gs.GS_F32)
    say("[noalloc] 2D J=5 M=3000")
    _check(gs, small, to_dev(crandn(rng, 3000), torch.complex64), 0, torch.complex64)
    one = gs.gs_plan(1, 9, 3, rng.uniform(-300, 300, 2000), rng.uniform(0.5, 2, 2000), precision=gs.GS_F64)
    say("[noalloc] 1D J=9 M=2000 sorted")
    _check(gs, one, to_dev(crandn(rng, 2000), torch.complex128), gs.GS_WEIGHTED | gs.GS_SORTED, torch.complex128)
    for pl in (big, small, one):
        pl.destroy()


def test_noalloc_refuses_oversized_workspace(gs):
    # a 2048^2 FP64 grid alone is 64 MiB
    rng = np.random.default_rng(8)
    plan = gs.gs_plan(2, 10, 2, rng.uniform(-500, 500, (1000, 2)), None, precision=gs.GS_F64)
    u = to_dev(crandn(rng, 1000), torch.complex128)
    x = torch.zeros(plan.coef_shape(), dtype=torch.complex128, device="cuda")
    say("[noalloc] oversized")
    assert _noalloc(gs, plan, u, x, 0) == gs.GS_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert float(torch.abs(x).max()) == 0.0      # nothing ran
    plan.destroy()
