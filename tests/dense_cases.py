"""Input recipes of the dense full-size adjoint checks (no method arithmetic).

Each case fixes a point set, weights, a DENSE random input u over every point
and a list of sampled output coefficients.  tests/golden/make_dense_golden.py
forms the oracle's value of each sampled coefficient of T^H (W^{1/2}) u from
these inputs; the GPU tests rebuild the same inputs from the same seeds, run
the full adjoint, and compare the sampled coefficients with the stored values.
"""
import numpy as np

from workloads import config_c2, spiral_2d


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _sample_2d(N, seed, n_random=20):
    """12 fixed coefficients (corners, edges, boundary/interior seams, centre)
    and n_random seeded ones."""
    fixed = [(0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1), (3, 4), (4, N // 2 - 1), (N // 2, N // 2 + 1),
             (N - 4, 3), (N // 5, 4 * N // 5), (N // 2, 7), (2, 3 * N // 5), (N - 3, N - 2)]
    rng = np.random.default_rng(seed)
    extra = [tuple(int(v) for v in rng.integers(0, N, 2)) for _ in range(n_random)]
    return np.array(fixed + extra, dtype=np.int64)


def _sample_1d(N, seed, n_random=20):
    fixed = [0, 1, 2, 3, 4, 5, N // 2 - 1, N // 2, N - 6, N - 5, N - 4, N - 3, N - 2, N - 1]
    rng = np.random.default_rng(seed)
    return np.array(fixed + [int(v) for v in rng.integers(0, N, n_random)], dtype=np.int64)


def case(name):
    """dict(dim, J, p, xi, mu (None = unweighted), u, idx)."""
    if name in ("spiral_1M_J9", "spiral_262k_J8"):
        J, per_arm, r_max = (9, 16384, 256.0) if name == "spiral_1M_J9" else (8, 4096, 128.0)
        pts = spiral_2d(64, per_arm, r_max, 0.5)
        M = pts.shape[0]
        mu = np.random.default_rng(2024).uniform(0.5, 1.5, M)
        u = crandn(np.random.default_rng(14), M)
        return dict(dim=2, J=J, p=4, xi=pts, mu=mu, u=u, idx=_sample_2d(1 << J, 15))
    if name == "limits_2d_J11":
        J, p, M = 11, 2, 100_000
        N = 1 << J
        pts = np.random.default_rng(111).uniform(-N, N, (M, 2))
        u = crandn(np.random.default_rng(116), M)
        return dict(dim=2, J=J, p=p, xi=pts, mu=None, u=u, idx=_sample_2d(N, 118))
    if name == "limits_1d_J20":
        J, p, M = 20, 4, 1_000_000
        N = 1 << J
        xi = np.random.default_rng(112).uniform(-N, N, M)
        u = crandn(np.random.default_rng(117), M)
        return dict(dim=1, J=J, p=p, xi=xi, mu=None, u=u, idx=_sample_1d(N, 119))
    if name == "c2_J14":
        c = config_c2()
        u = crandn(np.random.default_rng(23), c["xi"].size)
        return dict(dim=1, J=14, p=4, xi=c["xi"], mu=c["mu"], u=u, idx=_sample_1d(1 << 14, 24))
    raise KeyError(name)


NAMES = ["spiral_1M_J9", "spiral_262k_J8", "limits_2d_J11", "limits_1d_J20", "c2_J14"]


def load_expected(name):
    """Stored oracle values of the sampled coefficients (complex128)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dense_adjoint_samples.json")
    with open(path) as f:
        d = json.load(f)[name]
    return np.array(d["re"]) + 1j * np.array(d["im"])
