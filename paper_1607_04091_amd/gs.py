"""Thin ctypes binding of libgs.so (the C ABI declared in include/gs.h).

Argument marshalling only: every step of T, T^H and the CGLS solve runs in the
library's HIP kernels.  Device vectors are torch tensors on a ROCm device
(complex128 for FP64 data, complex64 for FP32 data); host arrays are numpy.
If the library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GS_LIB", os.path.join(_HERE, "lib", "libgs.so"))

GS_OK = 0
GS_NOT_CONVERGED = 1
GS_ERR_INVALID_ARG = -1
GS_ERR_UNSUPPORTED = -2
GS_ERR_BAD_NODES = -3
GS_ERR_NOMEM = -4
GS_ERR_HIP = -5
GS_ERR_BREAKDOWN = -6
GS_ERR_PRECISION = -7
GS_ERR_TOO_LARGE = -8
GS_NOALLOC_SCRATCH_BYTES = 64 << 20

GS_F64, GS_F32, GS_F32_MIXED = 0, 1, 2
GS_WEIGHTED, GS_SORTED, GS_APPLY_F64, GS_WEIGHT_FULL = 1, 2, 4, 8


def _wflags(weighted):
    """weighted: False, True (W^{1/2}) or "full" (W)."""
    if weighted == "full":
        return GS_WEIGHTED | GS_WEIGHT_FULL
    return GS_WEIGHTED if weighted else 0

EXPORTS = [
    "gs_plan", "gs_plan_batch", "gs_apply_T", "gs_apply_TH", "gs_apply_TH_noalloc", "gs_solve", "gs_solve_batch", "gs_destroy", "gs_get_plan_info",
    "gs_get_permutation", "gs_get_channels", "gs_weval", "gs_strerror", "gs_version", "gs_filter_taps", "gs_boundary_filters",
    "gs_eval_basis_1d", "gs_profile_enable", "gs_profile_read",
    "gs_cnn_param_count", "gs_cnn_create", "gs_cnn_destroy", "gs_cnn_set_weights", "gs_cnn_get_weights",
    "gs_cnn_get_grads", "gs_cnn_get_state", "gs_cnn_set_state", "gs_cnn_forward", "gs_cnn_backward", "gs_cnn_step",
    "gs_cnn_set_input_scale", "gs_cnn_get_input_scale",
]

GS_CNN_IN_F64, GS_CNN_OUT_F64, GS_CNN_TRAIN, GS_CNN_TGT_F64 = 1, 2, 4, 8


class GSError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


class SolveOpts(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("refine_fp64", ctypes.c_int), ("max_restarts", ctypes.c_int), ("check_every", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("rel_residual_fp64", ctypes.c_double),
                ("warm_start_used", ctypes.c_int), ("batch_class", ctypes.c_int), ("batch_streams", ctypes.c_int)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("J", ctypes.c_int), ("p", ctypes.c_int), ("precision", ctypes.c_int),
                ("M", ctypes.c_int64), ("xi", ctypes.POINTER(ctypes.c_double)),
                ("mu", ctypes.POINTER(ctypes.c_double))]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("J", ctypes.c_int), ("p", ctypes.c_int), ("N", ctypes.c_int),
                ("precision", ctypes.c_int), ("M", ctypes.c_int64), ("grid_n", ctypes.c_int),
                ("window_w32", ctypes.c_int), ("window_w64", ctypes.c_int), ("device_bytes", ctypes.c_int64),
                ("exact_nodes", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgs.so not built ({LIB_PATH}); run python -m paper_1607_04091_amd.build")
    # torch ships its own HIP runtime with the same SONAME as the system one.
    # Loading torch first makes libgs bind to that single runtime; loading
    # libgs first would bring a second HIP/HSA runtime into the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.gs_plan.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i64, dp, dp, i32, vp]
    lib.gs_plan_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(PlanDesc), vp]
    lib.gs_apply_T.argtypes = [vp, vp, vp, i32, vp]
    lib.gs_apply_TH.argtypes = [vp, vp, vp, i32, vp]
    lib.gs_apply_TH_noalloc.argtypes = [vp, vp, vp, i32, vp]
    lib.gs_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    lib.gs_solve_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), i32, vp]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.gs_cnn_param_count.argtypes = []
    lib.gs_cnn_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32]
    lib.gs_cnn_destroy.argtypes = [vp]
    lib.gs_cnn_destroy.restype = None
    lib.gs_cnn_set_weights.argtypes = [vp, fp]
    lib.gs_cnn_get_weights.argtypes = [vp, fp]
    lib.gs_cnn_get_grads.argtypes = [vp, fp]
    lib.gs_cnn_get_state.argtypes = [vp, fp, fp, ctypes.POINTER(ctypes.c_int)]
    lib.gs_cnn_set_state.argtypes = [vp, fp, fp, i32]
    lib.gs_cnn_forward.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.gs_cnn_backward.argtypes = [vp, vp, i32, i32, dp, vp]
    lib.gs_cnn_set_input_scale.argtypes = [vp, ctypes.c_float]
    lib.gs_cnn_get_input_scale.argtypes = [vp, fp]
    lib.gs_cnn_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    lib.gs_destroy.argtypes = [vp]
    lib.gs_destroy.restype = None
    lib.gs_get_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.gs_get_permutation.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.gs_get_channels.argtypes = [vp, i32, i32, vp]
    lib.gs_weval.argtypes = [i32, i32, i32, i32, vp, vp, vp]
    lib.gs_strerror.argtypes = [i32]
    lib.gs_strerror.restype = ctypes.c_char_p
    lib.gs_version.argtypes = []
    lib.gs_filter_taps.argtypes = [i32, dp]
    lib.gs_boundary_filters.argtypes = [i32, dp, dp, dp, dp, dp, dp]
    lib.gs_eval_basis_1d.argtypes = [i32, i32, i64, dp, dp]
    lib.gs_profile_enable.argtypes = [i32]
    lib.gs_profile_read.argtypes = [i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), dp,
                                    ctypes.POINTER(ctypes.c_int)]
    return lib


_lib = _load()


def library():
    return _lib


def strerror(code: int) -> str:
    return _lib.gs_strerror(int(code)).decode()


def gs_version() -> int:
    return _lib.gs_version()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _is_device_tensor(t) -> bool:
    return bool(getattr(t, "is_cuda", False))


def _check_vec(t, dtype, numel, name, like=None):
    """Validates a device vector handed to the library (input or output):
    element type, element count, contiguity, and that it lives on a GPU (the
    same one as `like`, if given).  Raises ValueError before any library call,
    so a wrong buffer never reaches a kernel."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not _is_device_tensor(t):
        raise ValueError(f"{name} must be a GPU tensor")
    if like is not None and t.device != like.device:
        raise ValueError(f"{name} must be on {like.device}, got {t.device}")


# ------------------------------------------------------------------ per-kernel timing

def gs_profile_enable(enable: bool = True):
    rc = _lib.gs_profile_enable(int(enable))
    if rc:
        raise GSError(rc, "gs_profile_enable")


def gs_profile_read() -> dict:
    """{kernel name: (launch count, total ms)} since the last enable."""
    nmax = 64
    names = ctypes.create_string_buffer(32 * nmax)
    counts = (ctypes.c_int64 * nmax)()
    tot = (ctypes.c_double * nmax)()
    n = ctypes.c_int(0)
    rc = _lib.gs_profile_read(nmax, names, counts, tot, ctypes.byref(n))
    if rc:
        raise GSError(rc, "gs_profile_read")
    raw = names.raw
    out = {}
    for i in range(n.value):
        nm = raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (int(counts[i]), float(tot[i]))
    return out


# ------------------------------------------------------------------ host-only queries

def gs_filter_taps(p: int) -> np.ndarray:
    h = np.zeros(2 * p)
    rc = _lib.gs_filter_taps(p, _dptr(h))
    if rc:
        raise GSError(rc, "gs_filter_taps")
    return h


def gs_boundary_filters(p: int):
    out = [np.zeros((p, p)), np.zeros((p, 2 * p - 1)), np.zeros(p),
           np.zeros((p, p)), np.zeros((p, 2 * p - 1)), np.zeros(p)]
    rc = _lib.gs_boundary_filters(p, *[_dptr(a) for a in out])
    if rc:
        raise GSError(rc, "gs_boundary_filters")
    return {"U_left": out[0], "V_left": out[1], "v0_left": out[2],
            "U_right": out[3], "V_right": out[4], "v0_right": out[5]}


def gs_eval_basis_1d(J: int, p: int, xi) -> np.ndarray:
    """(M, 2nb+1) complex128: [left boundary cols, D, right boundary cols]."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    nb = 0 if p == 1 else p
    out = np.zeros((xi.size, 2 * nb + 1), dtype=np.complex128)
    rc = _lib.gs_eval_basis_1d(J, p, xi.size, _dptr(xi), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise GSError(rc, "gs_eval_basis_1d")
    return out


# ------------------------------------------------------------------ evaluation in space

def gs_weval(coef, J: int, p: int, R: int, out=None, stream=None):
    """f on the dyadic grid x_j = -1/2 + j 2^-R (j = 0..2^R) from the
    coefficients (a complex128 GPU tensor of shape (N,) or (N, N)); returns
    (x as a numpy array, f as a complex128 GPU tensor of shape (2^R+1,)^dim)."""
    import torch
    dim = coef.dim()
    N = 1 << J
    if dim not in (1, 2):
        raise ValueError("coef must be 1D or 2D")
    _check_vec(coef, torch.complex128, N ** dim, "coef")
    side = (1 << R) + 1
    if out is None:
        out = torch.empty((side,) * dim, dtype=torch.complex128, device=coef.device)
    _check_vec(out, torch.complex128, side ** dim, "out", like=coef)
    rc = _lib.gs_weval(dim, J, p, R, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                       _stream(stream))
    if rc:
        raise GSError(rc, "gs_weval")
    return np.arange(side) / (1 << R) - 0.5, out


# ------------------------------------------------------------------ plans

def gs_plan(dim: int, J: int, p: int, xi, mu=None, precision: int = GS_F64, stream=None) -> "Plan":
    """Build a plan (the paper's Freq2Wave init).  xi: (M,) or (M, 2) host array."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    M = xi.shape[0]
    mu_a = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = _lib.gs_plan(ctypes.byref(h), dim, J, p, M, _dptr(xi),
                      None if mu_a is None else _dptr(mu_a), precision,
                      ctypes.c_void_p(0) if stream is None else _stream(stream))
    if rc:
        raise GSError(rc, "gs_plan")
    return Plan(h, dim, J, p, M, precision)


def gs_plan_batch(descs, stream=None) -> list:
    """Plans of many problems in one call (all or nothing).  descs: a sequence of
    dicts with the keys dim, J, p, xi and optionally mu, precision (as gs_plan)."""
    n = len(descs)
    if n < 1:
        raise ValueError("gs_plan_batch: no descriptors")
    arr = (PlanDesc * n)()
    keep = []
    for i, d in enumerate(descs):
        xi = np.ascontiguousarray(d["xi"], dtype=np.float64)
        mu = d.get("mu")
        mu_a = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
        if mu_a is not None and mu_a.size != xi.shape[0]:
            raise ValueError(f"gs_plan_batch: descriptor {i}: {mu_a.size} weights for {xi.shape[0]} points")
        keep += [xi, mu_a]
        arr[i] = PlanDesc(d["dim"], d["J"], d["p"], d.get("precision", GS_F64), xi.shape[0], _dptr(xi),
                          None if mu_a is None else _dptr(mu_a))
    hs = (ctypes.c_void_p * n)()
    rc = _lib.gs_plan_batch(hs, n, arr, ctypes.c_void_p(0) if stream is None else _stream(stream))
    if rc:
        raise GSError(rc, "gs_plan_batch")
    return [Plan(ctypes.c_void_p(hs[i]), d["dim"], d["J"], d["p"], int(arr[i].M), int(arr[i].precision))
            for i, d in enumerate(descs)]


class Plan:
    def __init__(self, handle, dim, J, p, M, precision):
        self._h = handle
        self.dim, self.J, self.p, self.M, self.precision = dim, J, p, M, precision
        self.N = 1 << J

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("plan destroyed")
        return self._h

    def info(self) -> dict:
        pi = PlanInfo()
        rc = _lib.gs_get_plan_info(self.handle, ctypes.byref(pi))
        if rc:
            raise GSError(rc, "gs_get_plan_info")
        return {f: getattr(pi, f) for f, _ in PlanInfo._fields_}

    def permutation(self) -> np.ndarray:
        out = np.zeros(self.M, dtype=np.int32)
        rc = _lib.gs_get_permutation(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if rc:
            raise GSError(rc, "gs_get_permutation")
        return out

    def channels(self, dimension=0, f64=True) -> np.ndarray:
        """The per-point basis table of one dimension, (2nb+1, M) complex, in
        the plan's internal point order."""
        nch = 2 * (0 if self.p == 1 else self.p) + 1
        out = np.zeros((nch, self.M), dtype=np.complex128 if f64 else np.complex64)
        rc = _lib.gs_get_channels(self.handle, int(dimension), int(bool(f64)), out.ctypes.data_as(ctypes.c_void_p))
        if rc:
            raise GSError(rc, "gs_get_channels")
        return out

    def coef_shape(self):
        return (self.N, self.N) if self.dim == 2 else (self.N,)

    def _dtype(self, f64: bool):
        import torch
        use64 = self.precision == GS_F64 or f64
        return torch.complex128 if use64 else torch.complex64

    def apply_T(self, x, y=None, weighted=False, sorted_order=False, f64=False, stream=None):
        import torch
        dt = self._dtype(f64)
        _check_vec(x, dt, self.N ** self.dim, "x")
        if y is None:
            y = torch.empty(self.M, dtype=dt, device=x.device)
        _check_vec(y, dt, self.M, "y", like=x)
        flags = _wflags(weighted) | (GS_SORTED if sorted_order else 0) | (GS_APPLY_F64 if f64 else 0)
        rc = _lib.gs_apply_T(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), flags,
                             _stream(stream))
        if rc:
            raise GSError(rc, "gs_apply_T")
        return y

    def apply_TH(self, u, x=None, weighted=False, sorted_order=False, f64=False, stream=None):
        import torch
        dt = self._dtype(f64)
        _check_vec(u, dt, self.M, "u")
        if x is None:
            x = torch.empty(self.coef_shape(), dtype=dt, device=u.device)
        _check_vec(x, dt, self.N ** self.dim, "x", like=u)
        flags = _wflags(weighted) | (GS_SORTED if sorted_order else 0) | (GS_APPLY_F64 if f64 else 0)
        rc = _lib.gs_apply_TH(self.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(x.data_ptr()), flags,
                              _stream(stream))
        if rc:
            raise GSError(rc, "gs_apply_TH")
        return x

    def apply_TH_noalloc(self, u, x, weighted=False, sorted_order=False, f64=False, stream=None):
        """gs_apply_TH_noalloc: the adjoint on the library's static device
        workspace; x (the output) must be supplied."""
        dt = self._dtype(f64)
        _check_vec(u, dt, self.M, "u")
        _check_vec(x, dt, self.N ** self.dim, "x", like=u)
        flags = _wflags(weighted) | (GS_SORTED if sorted_order else 0) | (GS_APPLY_F64 if f64 else 0)
        rc = _lib.gs_apply_TH_noalloc(self.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      flags, _stream(stream))
        if rc:
            raise GSError(rc, "gs_apply_TH_noalloc")
        return x

    def solve(self, y, x=None, rel_tol=1e-6, max_iter=500, warm_start=False, refine_fp64=True, max_restarts=2,
              check_every=1, history=False, stream=None):
        import torch
        _check_vec(y, torch.complex128, self.M, "y")
        if x is None:
            if warm_start:
                raise ValueError("warm_start needs x")
            x = torch.zeros(self.coef_shape(), dtype=torch.complex128, device=y.device)
        _check_vec(x, torch.complex128, self.N ** self.dim, "x", like=y)
        hist = np.zeros(max_iter + 1) if history else None
        # warm_start: False (x0 = 0), True (x holds x0) or "guarded" (x0 kept only if it beats x0 = 0)
        ws = 2 if warm_start == "guarded" else int(bool(warm_start))
        o = SolveOpts(rel_tol, max_iter, ws, int(refine_fp64), max_restarts, check_every,
                      _dptr(hist) if hist is not None else None, hist.size if hist is not None else 0)
        info = SolveInfo()
        rc = _lib.gs_solve(self.handle, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                           ctypes.byref(o), ctypes.byref(info), _stream(stream))
        if rc < 0:
            raise GSError(rc, "gs_solve")
        res = {"status": rc, "iterations": info.iterations, "restarts": info.restarts,
               "rel_residual": info.rel_residual, "rel_residual_fp64": info.rel_residual_fp64,
               "warm_start_used": bool(info.warm_start_used)}
        if hist is not None:
            res["history"] = hist[: info.iterations + 1].copy()
        return x, res

    def destroy(self):
        if self._h:
            _lib.gs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def gs_apply_T(plan: Plan, x, y=None, **kw):
    return plan.apply_T(x, y, **kw)


def gs_apply_TH(plan: Plan, u, x=None, **kw):
    return plan.apply_TH(u, x, **kw)


def gs_solve(plan: Plan, y, x=None, **kw):
    return plan.solve(y, x, **kw)


def gs_solve_batch(plans, ys, xs=None, rel_tol=1e-6, max_iter=500, refine_fp64=True, max_restarts=2,
                   check_every=1, n_streams=0, stream=None):
    """Solves len(plans) independent problems together (graph-captured CGLS
    iterations over several streams).  ys[i]: contiguous complex128 of length
    plans[i].M; xs[i] (optional): complex128 coefficient arrays, zero-started.
    Returns (xs, list of per-problem result dicts)."""
    import torch
    n = len(plans)
    if n < 1 or len(ys) != n:
        raise ValueError("need one y per plan")
    for p, y in zip(plans, ys):
        _check_vec(y, torch.complex128, p.M, "y[i]")
    if xs is None:
        xs = [torch.zeros(p.coef_shape(), dtype=torch.complex128, device=y.device) for p, y in zip(plans, ys)]
    if len(xs) != n:
        raise ValueError("need one x per plan")
    for p, y, x in zip(plans, ys, xs):
        _check_vec(x, torch.complex128, p.N ** p.dim, "x[i]", like=y)
    vp = ctypes.c_void_p
    hp = (vp * n)(*[p.handle for p in plans])
    yp = (vp * n)(*[y.data_ptr() for y in ys])
    xp = (vp * n)(*[x.data_ptr() for x in xs])
    o = SolveOpts(rel_tol, max_iter, 0, int(refine_fp64), max_restarts, check_every, None, 0)
    infos = (SolveInfo * n)()
    rc = _lib.gs_solve_batch(hp, n, yp, xp, ctypes.byref(o), infos, n_streams, _stream(stream))
    if rc < 0:
        raise GSError(rc, "gs_solve_batch")
    res = [{"status": i.status, "iterations": i.iterations, "restarts": i.restarts,
            "rel_residual": i.rel_residual, "rel_residual_fp64": i.rel_residual_fp64,
            "warm_start_used": bool(i.warm_start_used), "batch_class": i.batch_class,
            "batch_streams": i.batch_streams} for i in infos]
    return xs, res


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Cnn:
    """The learned warm start network (see include/gs.h): a handle for
    images of height x width and batches up to max_batch."""

    def __init__(self, height, width, max_batch=1):
        h = ctypes.c_void_p()
        rc = _lib.gs_cnn_create(ctypes.byref(h), int(height), int(width), int(max_batch))
        if rc:
            raise GSError(rc, "gs_cnn_create")
        self._h = h.value
        self.height, self.width, self.max_batch = int(height), int(width), int(max_batch)
        self.n_params = _lib.gs_cnn_param_count()

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("network destroyed")
        return self._h

    def _check(self, rc, where):
        if rc:
            raise GSError(rc, where)

    def set_weights(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"need {self.n_params} parameters")
        self._check(_lib.gs_cnn_set_weights(self.handle, _fptr(a)), "gs_cnn_set_weights")

    def _get(self, fn, where):
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(fn(self.handle, _fptr(a)), where)
        return a

    def get_weights(self):
        return self._get(_lib.gs_cnn_get_weights, "gs_cnn_get_weights")

    def get_grads(self):
        return self._get(_lib.gs_cnn_get_grads, "gs_cnn_get_grads")

    @property
    def input_scale(self):
        s = ctypes.c_float()
        self._check(_lib.gs_cnn_get_input_scale(self.handle, ctypes.byref(s)), "gs_cnn_get_input_scale")
        return s.value

    @input_scale.setter
    def input_scale(self, s):
        self._check(_lib.gs_cnn_set_input_scale(self.handle, float(s)), "gs_cnn_set_input_scale")

    def get_state(self):
        m = np.empty(self.n_params, dtype=np.float32)
        v = np.empty(self.n_params, dtype=np.float32)
        st = ctypes.c_int()
        self._check(_lib.gs_cnn_get_state(self.handle, _fptr(m), _fptr(v), ctypes.byref(st)), "gs_cnn_get_state")
        return m, v, st.value

    def set_state(self, m, v, step):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        self._check(_lib.gs_cnn_set_state(self.handle, _fptr(m), _fptr(v), int(step)), "gs_cnn_set_state")

    def _images(self, x, name):
        import torch
        if x.dtype not in (torch.complex64, torch.complex128) or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex64 or complex128 tensor")
        if x.dim() == 2:
            x = x.unsqueeze(0)
        if x.dim() != 3 or tuple(x.shape[1:]) != (self.height, self.width):
            raise ValueError(f"{name} must have shape (batch, {self.height}, {self.width})")
        if not 1 <= x.shape[0] <= self.max_batch:
            raise ValueError(f"{name} must hold 1..{self.max_batch} images")
        if not _is_device_tensor(x):
            raise ValueError(f"{name} must be a GPU tensor")
        return x

    def forward(self, x, out=None, train=False, out_dtype=None, stream=None):
        import torch
        squeeze = x.dim() == 2
        x = self._images(x, "x")
        if out is None and not (train and out_dtype is None):
            out = torch.empty(x.shape, dtype=out_dtype or x.dtype, device=x.device)
        if out is not None:
            out = self._images(out, "out")
            if out.shape[0] != x.shape[0]:
                raise ValueError(f"out holds {out.shape[0]} images, x {x.shape[0]}")
            if not _is_device_tensor(out) or out.device != x.device:
                raise ValueError(f"out must be on {x.device}")
        flags = (GS_CNN_IN_F64 if x.dtype == torch.complex128 else 0) | (GS_CNN_TRAIN if train else 0)
        if out is not None and out.dtype == torch.complex128:
            flags |= GS_CNN_OUT_F64
        rc = _lib.gs_cnn_forward(self.handle, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr() if out is not None else 0), x.shape[0], flags,
                                 _stream(stream))
        self._check(rc, "gs_cnn_forward")
        if out is None:
            return None
        return out[0] if squeeze else out

    def backward(self, target, stream=None, want_loss=True):
        import torch
        t = self._images(target, "target")
        flags = GS_CNN_TGT_F64 if t.dtype == torch.complex128 else 0
        loss = ctypes.c_double(float("nan"))
        rc = _lib.gs_cnn_backward(self.handle, ctypes.c_void_p(t.data_ptr()), t.shape[0], flags,
                                  ctypes.byref(loss) if want_loss else None, _stream(stream))
        self._check(rc, "gs_cnn_backward")
        return loss.value

    def step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(_lib.gs_cnn_step(self.handle, lr, beta1, beta2, eps, _stream(stream)), "gs_cnn_step")

    def save(self, path):
        m, v, step = self.get_state()
        np.savez(path, weights=self.get_weights(), m=m, v=v, step=np.int64(step),
                 input_scale=np.float32(self.input_scale),
                 shape=np.array([self.height, self.width], dtype=np.int64))

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.set_weights(z["weights"])
            if "input_scale" in z:
                self.input_scale = float(z["input_scale"])
            if "m" in z and "v" in z:
                self.set_state(z["m"], z["v"], int(z["step"]))

    def destroy(self):
        if self._h:
            _lib.gs_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def cnn_he_init(seed, last_scale=0.1):
    """He-normal initial weights (std sqrt(2 / (9 ci))) for the six layers,
    the last one scaled by last_scale, as the flat FP32 parameter array."""
    rng = np.random.default_rng(seed)
    ch = [2, 32, 32, 32, 32, 32, 2]
    parts = []
    for l in range(6):
        std = np.sqrt(2.0 / (9 * ch[l])) * (last_scale if l == 5 else 1.0)
        parts.append((rng.standard_normal((3, 3, ch[l], ch[l + 1])) * std).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def gs_destroy(plan: Plan):
    plan.destroy()
