"""Writes the stored oracle values used by the dense full-size checks.

* dense_adjoint_samples.json: for every case of tests/dense_cases.py, the
  sampled coefficients of T^H W^{1/2} u (T^H u when unweighted) for a dense
  random u over all points -- App. C for 2D (X[i,j] = sum_m conj(b_i(xi_x,m)
  b_j(xi_y,m)) w_m u_m), Sec. 4 for 1D (x_n = sum_m conj(b_n(xi_m)) w_m u_m) --
  with the columns b_n formed by oracle.basis.
* c2_y_oracle.npy: y = T x0 for the 65,536-point 1D workload (db4, J = 14),
  the oracle's dense rows applied to x0 (Sec. 4, eq. CoB_block_1D).

Calls only oracle/ (plus the seeded input recipes).  The point sums run over
chunks of points in a process pool; each chunk's sums are the plain products
of the oracle's columns.  Run from the repository root:
    python tests/golden/make_dense_golden.py [case ...]
"""
import json
import os
import sys
import time
from multiprocessing import Pool

# one BLAS thread per worker process: the pool provides the parallelism
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import basis  # noqa: E402
import dense_cases  # noqa: E402

CHUNK = 32768


def _partial(args):
    dim, J, p, xs, ys, wu, idx = args
    if dim == 2:
        bx = basis.columns_subset_1d(xs, J, p, idx[:, 0])
        by = basis.columns_subset_1d(ys, J, p, idx[:, 1])
        return np.array([np.sum(np.conj(bx[i] * by[j]) * wu) for i, j in idx])
    b = basis.columns_subset_1d(xs, J, p, idx)
    return np.array([np.sum(np.conj(b[n]) * wu) for n in idx])


def sampled_adjoint(c, workers):
    xi, u, idx = c["xi"], c["u"], c["idx"]
    wu = u * (np.sqrt(c["mu"]) if c["mu"] is not None else 1.0)
    M = u.size
    jobs = []
    for s in range(0, M, CHUNK):
        e = min(M, s + CHUNK)
        if c["dim"] == 2:
            jobs.append((2, c["J"], c["p"], xi[s:e, 0], xi[s:e, 1], wu[s:e], idx))
        else:
            jobs.append((1, c["J"], c["p"], xi[s:e], None, wu[s:e], idx))
    with Pool(workers) as pool:
        parts = pool.map(_partial, jobs)
    return np.sum(parts, axis=0)


def _rows(args):
    xs, J, p, x0 = args
    return basis.apply_T_1d(xs, J, p, x0, chunk=2048)


def c2_y(workers):
    from workloads import config_c2
    c = config_c2()
    xi = c["xi"]
    jobs = [(xi[s:s + 4096], 14, 4, c["x0"]) for s in range(0, xi.size, 4096)]
    with Pool(workers) as pool:
        parts = pool.map(_rows, jobs)
    return np.concatenate(parts)


def main(names):
    workers = min(8, os.cpu_count() or 1)
    path = os.path.join(HERE, "dense_adjoint_samples.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        if name == "c2_y":
            t = time.time()
            y = c2_y(workers)
            np.save(os.path.join(HERE, "c2_y_oracle.npy"), y)
            print(f"c2_y: {y.size} values, {time.time() - t:.0f} s", flush=True)
            continue
        t = time.time()
        c = dense_cases.case(name)
        v = sampled_adjoint(c, workers)
        out[name] = {"re": [float(a) for a in v.real], "im": [float(a) for a in v.imag],
                     "idx": c["idx"].tolist(), "M": int(c["u"].size)}
        print(f"{name}: {len(v)} coefficients, {time.time() - t:.0f} s", flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=0)


if __name__ == "__main__":
    main(sys.argv[1:] or dense_cases.NAMES + ["c2_y"])
