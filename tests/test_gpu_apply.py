"""Parity of the HIP T and T^H (through the C ABI) with the FP64 oracle's dense
products, element by element, on seeded inputs.  Tolerances: relative error
<= 1e-12 for FP64 applies and <= 2e-5 for FP32 applies."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis
from workloads import grid, jitter_1d, spiral_2d, jitter_2d, voronoi_weights_1d, voronoi_weights_2d

from gpu_util import assert_close, rel, crandn, to_dev, to_host, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-5}


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_04091_amd import gs as _gs
    return _gs


def _case_1d(J, p, M, kind, seed):
    rng = np.random.default_rng(seed)
    N = 1 << J
    if kind == "uniform":
        xi = grid(M, 0.5)
        mu = None
    elif kind == "jitter":
        xi = jitter_1d(M, N / M * 2.0, seed)
        mu = voronoi_weights_1d(xi, np.abs(xi).max() + 0.5)
    elif kind == "edges":  # grid nodes, band edges +-N, repeats
        xi = 0.25 * rng.integers(-4 * N, 4 * N + 1, M).astype(float)
        xi[:6] = [-N, N, 0.0, -0.0, N - 0.25, -N / 2]
        xi[6:9] = xi[0]
        mu = rng.uniform(0.1, 2.0, M)
    else:  # random, beyond the band and with repeated points
        xi = rng.uniform(-1.3 * N, 1.3 * N, M)
        xi[:5] = xi[min(5, M - 1)]
        mu = rng.uniform(0.1, 2.0, M)
    return xi, mu


ONE_D = [
    # J, p, M, kind
    (6, 2, 200, "random"),
    (8, 2, 1024, "uniform"),      # C1 shape
    (7, 4, 555, "jitter"),
    (5, 1, 301, "random"),        # Haar
    (9, 3, 1500, "random"),
    (12, 4, 6000, "jitter"),      # grid 8192 > LDS limit: four-step FFT
    (3, 4, 50, "random"),         # 2^J = 2p: no interior column
    (7, 3, 900, "edges"),         # nodes, band edges, repeats
    (6, 4, 1, "random"),          # a single point
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("J,p,M,kind", ONE_D)
def test_apply_1d(gs, J, p, M, kind, prec):
    say(f"[apply_1d] J={J} p={p} M={M} {kind} prec={prec}")
    xi, mu = _case_1d(J, p, M, kind, 1000 * J + p)
    rng = np.random.default_rng(7 + J)
    N = 1 << J
    x = crandn(rng, N)
    u = crandn(rng, M)
    T = basis.dense_T_1d(xi, J, p)
    plan = gs.gs_plan(1, J, p, xi, mu, precision=prec)
    dt = torch.complex128 if prec == 0 else torch.complex64
    y = to_host(plan.apply_T(to_dev(x, dt)))
    assert_close(y, T @ x, TOL[prec], "y")
    z = to_host(plan.apply_TH(to_dev(u, dt)))
    assert_close(z, T.conj().T @ u, TOL[prec], "z")
    if mu is not None:
        s = np.sqrt(mu)
        yw = to_host(plan.apply_T(to_dev(x, dt), weighted=True))
        assert_close(yw, s * (T @ x), TOL[prec], "yw")
        zw = to_host(plan.apply_TH(to_dev(u, dt), weighted=True))
        assert_close(zw, T.conj().T @ (s * u), TOL[prec], "zw")
    plan.destroy()


def _case_2d(J, p, kind, M, seed):
    N = 1 << J
    if kind == "spiral":
        arms = 16
        pts = spiral_2d(arms, max(1, M // arms), N / 2, 0.5 * 64 / arms)
        mu = voronoi_weights_2d(pts, "disk", N / 2 + 0.25, 0.4)
    elif kind == "jitter":
        pts = jitter_2d(M, N / 2, seed)
        mu = voronoi_weights_2d(pts, "square", N / 2, N / np.sqrt(M))
    elif kind == "cluster":
        # every point within 0.2 of one frequency: one or two grid cells, one tile
        # holding all M points (many staging chunks in one row block)
        rng = np.random.default_rng(seed)
        r = 0.2 * np.sqrt(rng.uniform(0, 1, M))
        a = rng.uniform(0, 2 * np.pi, M)
        pts = np.stack([0.37 * N + r * np.cos(a), -0.21 * N + r * np.sin(a)], axis=1)
        mu = rng.uniform(0.5, 1.5, M)
    elif kind == "edges":
        # points on grid nodes (zero fractional position), on the band edges +-N
        # (wrap to the same node as 0 in the oversampled grid) and a few repeats
        rng = np.random.default_rng(seed)
        k = rng.integers(-4 * N, 4 * N + 1, (M, 2))
        pts = 0.25 * k.astype(float)
        pts[:8] = [[-N, -N], [N, N], [-N, N], [N, -N], [0.0, -0.0], [-N / 2, N / 2], [N - 0.25, -N], [0.0, 0.0]]
        pts[8:12] = pts[4]
        mu = rng.uniform(0.5, 1.5, M)
    else:
        rng = np.random.default_rng(seed)
        pts = rng.uniform(-0.8 * N, 0.8 * N, (M, 2))
        mu = rng.uniform(0.5, 1.5, M)
    return pts, mu


TWO_D = [
    (4, 2, "random", 700),
    (5, 4, "spiral", 3000),
    (5, 1, "jitter", 2000),       # Haar
    (6, 3, "jitter", 9000),
    (3, 4, "random", 400),        # no interior
    (6, 4, "random", 5000),
    (7, 4, "random", 6000),       # 256^2 grid: two-pass register column transform (16 x 16)
    (8, 3, "spiral", 8000),       # 512^2 grid (32 x 16)
    (6, 4, "cluster", 3000),      # all points in one tile
    (5, 3, "edges", 1500),        # nodes, band edges, repeats
    (6, 4, "random", 1),          # a single point
    (7, 2, "random", 37),         # almost every tile empty
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("J,p,kind,M", TWO_D)
def test_apply_2d(gs, J, p, kind, M, prec):
    say(f"[apply_2d] J={J} p={p} {kind} M={M} prec={prec}")
    pts, mu = _case_2d(J, p, kind, M, 31 * J + p)
    M = pts.shape[0]
    N = 1 << J
    rng = np.random.default_rng(11 + J)
    X = crandn(rng, (N, N))
    u = crandn(rng, M)
    plan = gs.gs_plan(2, J, p, pts, mu, precision=prec)
    dt = torch.complex128 if prec == 0 else torch.complex64
    y = to_host(plan.apply_T(to_dev(X, dt)))
    assert_close(y, basis.apply_T_2d(pts, J, p, X), TOL[prec], "y")
    Z = to_host(plan.apply_TH(to_dev(u, dt)))
    assert_close(Z, basis.apply_TH_2d(pts, J, p, u), TOL[prec], "Z")
    s = np.sqrt(mu)
    yw = to_host(plan.apply_T(to_dev(X, dt), weighted=True))
    assert_close(yw, s * basis.apply_T_2d(pts, J, p, X), TOL[prec], "yw")
    Zw = to_host(plan.apply_TH(to_dev(u, dt), weighted=True))
    assert_close(Zw, basis.apply_TH_2d(pts, J, p, s * u), TOL[prec], "Zw")
    plan.destroy()


def test_adjoint_identity_and_determinism(gs):
    say("[adjoint/determinism]")
    pts, mu = _case_2d(6, 4, "spiral", 8000, 3)
    rng = np.random.default_rng(5)
    X = crandn(rng, (64, 64))
    u = crandn(rng, pts.shape[0])
    for prec, tol in ((0, 1e-13), (1, 1e-6)):
        plan = gs.gs_plan(2, 6, 4, pts, mu, precision=prec)
        dt = torch.complex128 if prec == 0 else torch.complex64
        Xd, ud = to_dev(X, dt), to_dev(u, dt)
        y = to_host(plan.apply_T(Xd))
        Z1 = plan.apply_TH(ud)
        Z2 = plan.apply_TH(ud)
        assert torch.equal(Z1, Z2)                         # bitwise reproducible, no atomics
        lhs = np.vdot(u, y)
        rhs = np.vdot(to_host(Z1), X)
        assert abs(lhs - rhs) / (np.linalg.norm(u) * np.linalg.norm(y)) < tol
        plan.destroy()


def test_sorted_order_and_permutation(gs):
    say("[sorted order]")
    xi, mu = _case_1d(7, 2, 400, "random", 9)
    plan = gs.gs_plan(1, 7, 2, xi, mu, precision=0)
    perm = plan.permutation()
    assert sorted(perm.tolist()) == list(range(400))
    rng = np.random.default_rng(1)
    x = to_dev(crandn(rng, 128), torch.complex128)
    y = to_host(plan.apply_T(x))
    ys = to_host(plan.apply_T(x, sorted_order=True))
    assert np.array_equal(ys, y[perm])
    u = crandn(rng, 400)
    z1 = to_host(plan.apply_TH(to_dev(u, torch.complex128)))
    z2 = to_host(plan.apply_TH(to_dev(u[perm], torch.complex128), sorted_order=True))
    assert np.array_equal(z1, z2)
    info = plan.info()
    assert info["grid_n"] == 256 and info["window_w64"] > 0 and info["device_bytes"] > 0
    plan.destroy()


def test_mixed_plan_has_both_paths(gs):
    say("[mixed plan]")
    pts, mu = _case_2d(5, 2, "random", 1500, 4)
    rng = np.random.default_rng(2)
    X = crandn(rng, (32, 32))
    plan = gs.gs_plan(2, 5, 2, pts, mu, precision=gs.GS_F32_MIXED)
    ref = basis.apply_T_2d(pts, 5, 2, X)
    y32 = to_host(plan.apply_T(to_dev(X, torch.complex64)))
    y64 = to_host(plan.apply_T(to_dev(X, torch.complex128), f64=True))
    assert_close(y32, ref, 2e-5, "y32")
    assert_close(y64, ref, 1e-12, "y64")
    plan32 = gs.gs_plan(2, 5, 2, pts, mu, precision=gs.GS_F32)
    with pytest.raises(gs.GSError):
        plan32.apply_T(to_dev(X, torch.complex128), f64=True)
    plan.destroy()
    plan32.destroy()


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("prec", [0, 2])
def test_full_weight_adjoint(gs, dim, prec):
    """GS_WEIGHT_FULL: T^H W u and W T x (the warm-start network's input
    A^H b = T^H W y), against the oracle's dense T with diag(mu)."""
    say(f"[full weight] dim={dim} prec={prec}")
    rng = np.random.default_rng(31 + dim)
    if dim == 1:
        J, p = 6, 3
        xi = rng.uniform(-40, 40, 300)
        T = basis.dense_T_1d(xi, J, p)
        shape = (1 << J,)
    else:
        J, p = 4, 2
        xi = rng.uniform(-9, 9, (500, 2))
        T = basis.dense_T_2d(xi, J, p)
        shape = (1 << J, 1 << J)
    mu = rng.uniform(0.2, 3.0, xi.shape[0])
    plan = gs.gs_plan(dim, J, p, xi, mu, precision=prec)
    f64 = prec == 2
    u = crandn(rng, xi.shape[0])
    x = crandn(rng, shape)
    got_adj = to_host(plan.apply_TH(to_dev(u, torch.complex128), weighted="full", f64=f64))
    got_fwd = to_host(plan.apply_T(to_dev(x, torch.complex128), weighted="full", f64=f64))
    assert_close(got_adj.reshape(-1), T.conj().T @ (mu * u), 1e-12, "T^H W u")
    assert_close(got_fwd, mu * (T @ x.reshape(-1)), 1e-12, "got_fwd")
    # the full-weight flag alone (without GS_WEIGHTED) is rejected
    import ctypes
    xin = to_dev(x, torch.complex128)
    yout = torch.empty(xi.shape[0], dtype=torch.complex128, device="cuda")
    rc = gs.library().gs_apply_T(plan.handle, ctypes.c_void_p(xin.data_ptr()), ctypes.c_void_p(yout.data_ptr()),
                                 gs.GS_WEIGHT_FULL | (gs.GS_APPLY_F64 if f64 else 0), None)
    assert rc == gs.GS_ERR_INVALID_ARG
    plan.destroy()


@pytest.mark.parametrize("dim,J,p,eps,n_per_dim", [(1, 8, 2, 0.5, 1024), (1, 7, 4, 0.25, 700), (1, 6, 3, 1.0, 200),
                                                   (2, 5, 4, 0.5, 64), (2, 4, 2, 0.25, 40), (2, 6, 1, 1.0, 64)])
@pytest.mark.parametrize("prec", [0, 1])
def test_uniform_nodes_exact_path(gs, dim, J, p, eps, n_per_dim, prec):
    """Frequencies on a grid eps Z (eps = 1, 1/2, 1/4; the paper's uniform
    case, Sec. 3.2): the plan takes the exact path (a zero-padded FFT read at
    the nodes, no window).  Against the dense oracle the FP64 error is then at
    the FFT's rounding level, well below the windowed NFFT's 8e-14; FP32 as
    usual.  The 1D C1 shape (db2, J = 8, 1024 points k/2) is the first case; the
    2D cases are full uniform grids (the paper's Uniform 2D pattern, smaller)."""
    say(f"[uniform] dim={dim} J={J} p={p} eps={eps} prec={prec}")
    N = 1 << J
    k = np.arange(n_per_dim) - n_per_dim // 2
    if dim == 1:
        xi = eps * k.astype(float)
        T = basis.dense_T_1d(xi, J, p)
        shape = (N,)
    else:
        KX, KY = np.meshgrid(k, k, indexing="ij")
        xi = eps * np.stack([KX.ravel(), KY.ravel()], axis=1).astype(float)
        T = basis.dense_T_2d(xi, J, p)
        shape = (N, N)
    M = xi.shape[0]
    rng = np.random.default_rng(90 + J)
    mu = rng.uniform(0.5, 1.5, M)
    plan = gs.gs_plan(dim, J, p, xi, mu, precision=prec)
    assert plan.info()["exact_nodes"] == 1
    dt = torch.complex128 if prec == 0 else torch.complex64
    x = crandn(rng, shape)
    u = crandn(rng, M)
    tol = 1e-14 if prec == 0 else 2e-5
    s = np.sqrt(mu)
    assert_close(to_host(plan.apply_T(to_dev(x, dt), weighted=True)), s * (T @ x.reshape(-1)), tol, "W^1/2 T x")
    assert_close(to_host(plan.apply_TH(to_dev(u, dt), weighted=True)).reshape(-1), T.conj().T @ (s * u), tol,
                 "T^H W^1/2 u")
    plan.destroy()
    # one point off the grid: the windowed NFFT path
    xi2 = xi.copy()
    xi2[0] = xi2[0] + 1e-3
    plan2 = gs.gs_plan(dim, J, p, xi2, mu, precision=prec)
    assert plan2.info()["exact_nodes"] == 0
    plan2.destroy()


@pytest.mark.parametrize("dim,J,p,M", [(2, 9, 4, 200_000), (1, 14, 4, 65_536), (2, 6, 8, 3000), (1, 20, 3, 5000),
                                       (2, 5, 1, 2000), (1, 4, 2, 300)])
def test_device_plan_tables(gs, dim, J, p, M):
    """The plan's per-point tables are built on the device: they must equal
    the host evaluation (gs_eval_basis_1d, App. A product and App. A.1
    recursion) to 1e-14 in FP64, the FP32 tables must be the FP64 ones rounded,
    and the permutation must be the stable sort by cell (tile-major in 2D)."""
    say(f"[device plan] dim={dim} J={J} p={p} M={M}")
    rng = np.random.default_rng(500 + J + p)
    N = 1 << J
    xi = rng.uniform(-1.2 * N, 1.2 * N, (M, 2) if dim == 2 else M)
    xi[:3] = xi[3]                                  # repeated points keep their input order
    plan = gs.gs_plan(dim, J, p, xi, rng.uniform(0.5, 2, M), precision=gs.GS_F32_MIXED if J <= 14 else gs.GS_F64)
    perm = plan.permutation()
    assert np.array_equal(np.sort(perm), np.arange(M))
    # stable sort by cell: the key of the wrapped node, points of a cell in input order
    ng = max(2 * N, 16)
    cells = np.floor((np.asarray(xi).reshape(M, dim) / N % 1.0) * ng).astype(np.int64) % ng
    if dim == 2:
        ts = min(32, ng)
        ntx = ng // ts
        key = ((cells[:, 0] // ts) * ntx + cells[:, 1] // ts) * ts * ts + (cells[:, 0] % ts) * ts + cells[:, 1] % ts
    else:
        key = cells[:, 0]
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    for d in range(dim):
        x = np.asarray(xi).reshape(M, dim)[perm, d]
        host = gs.gs_eval_basis_1d(J, p, x).T          # (nch, M)
        dev64 = plan.channels(d, f64=True)
        assert np.max(np.abs(dev64 - host)) <= 1e-14 * np.max(np.abs(host)), np.max(np.abs(dev64 - host))
        if J <= 14:
            dev32 = plan.channels(d, f64=False)
            assert np.array_equal(dev32, dev64.astype(np.complex64))
    plan.destroy()
