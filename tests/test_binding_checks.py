"""CPU-only: the Python binding validates every device vector it hands to the
library -- inputs and caller-supplied outputs alike -- and raises ValueError
before any call into libgs.  A wrong buffer (element type, element count,
layout, device) would otherwise be written past its end by a kernel.

The library handle is replaced by a stub that fails the test if any entry
point is reached, and the device test is relaxed to accept CPU tensors (there
is no GPU here), so each case isolates one check."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1607_04091_amd import gs


class _NoCall:
    def __getattr__(self, name):
        def fail(*a, **k):
            raise AssertionError(f"library entry point {name} reached")
        return fail


@pytest.fixture
def stubbed(monkeypatch):
    monkeypatch.setattr(gs, "_lib", _NoCall())
    monkeypatch.setattr(gs, "_is_device_tensor", lambda t: True)
    yield


class _FakePlan(gs.Plan):
    """A plan object over a dummy handle; never released through the library."""

    def destroy(self):
        self._h = None


def _plan(dim=2, J=3, M=10, precision=gs.GS_F64):
    return _FakePlan(ctypes.c_void_p(0x1000), dim, J, 2, M, precision)


C128, C64 = torch.complex128, torch.complex64


def _z(n, dt=C128):
    return torch.zeros(n, dtype=dt)


@pytest.mark.parametrize("bad", ["dtype", "short", "long", "strided"])
def test_apply_outputs_rejected(stubbed, bad):
    p = _plan()
    x = torch.zeros((8, 8), dtype=C128)
    u = _z(10)

    def mk(n):
        if bad == "dtype":
            return _z(n, C64)
        if bad == "short":
            return _z(n - 1)
        if bad == "long":
            return _z(n + 1)
        return torch.zeros(2 * n, dtype=C128)[::2]

    with pytest.raises(ValueError):
        p.apply_T(x, y=mk(10))
    with pytest.raises(ValueError):
        p.apply_TH(u, x=mk(64))


def test_apply_inputs_rejected(stubbed):
    p = _plan(precision=gs.GS_F32)
    with pytest.raises(ValueError):
        p.apply_T(torch.zeros((8, 8), dtype=C128))        # FP32 plan takes complex64
    with pytest.raises(ValueError):
        p.apply_TH(_z(9, C64))                              # M = 10
    with pytest.raises(ValueError):
        p.apply_T(torch.zeros((8, 8), dtype=C64), f64=True, y=_z(10, C64))  # f64 wants complex128 IO


def test_solve_buffers_rejected(stubbed):
    p = _plan()
    y = _z(10)
    with pytest.raises(ValueError):
        p.solve(y, x=torch.zeros((8, 8), dtype=C64))        # x must be complex128
    with pytest.raises(ValueError):
        p.solve(y, x=_z(63))
    with pytest.raises(ValueError):
        p.solve(_z(10, C64))
    with pytest.raises(ValueError):
        p.solve(y, warm_start=True)                         # warm start needs x


def test_batch_buffers_rejected(stubbed):
    plans = [_plan(), _plan(J=4, M=12)]
    ys = [_z(10), _z(12)]
    with pytest.raises(ValueError):
        gs.gs_solve_batch(plans, ys, xs=[torch.zeros((8, 8), dtype=C128), torch.zeros((8, 8), dtype=C128)])
    with pytest.raises(ValueError):
        gs.gs_solve_batch(plans, ys, xs=[torch.zeros((8, 8), dtype=C128)])
    with pytest.raises(ValueError):
        gs.gs_solve_batch(plans, [_z(10), _z(11)])


def test_device_required(monkeypatch):
    """Without the relaxation, CPU tensors are refused before any call."""
    monkeypatch.setattr(gs, "_lib", _NoCall())
    p = _plan()
    with pytest.raises(ValueError, match="GPU"):
        p.apply_T(torch.zeros((8, 8), dtype=C128), y=_z(10))


def test_cnn_out_batch_rejected(stubbed):
    class _FakeCnn(gs.Cnn):
        def destroy(self):
            self._h = None

    net = _FakeCnn.__new__(_FakeCnn)
    net._h = 0x1000
    net.height, net.width, net.max_batch, net.n_params = 4, 5, 3, 38016
    x = torch.zeros((2, 4, 5), dtype=C64)
    with pytest.raises(ValueError):
        net.forward(x, out=torch.zeros((1, 4, 5), dtype=C64))
    with pytest.raises(ValueError):
        net.forward(torch.zeros((4, 4, 5), dtype=C64))      # above max_batch
    with pytest.raises(ValueError):
        net.forward(x, out=torch.zeros((2, 4, 6), dtype=C64))
