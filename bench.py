#!/usr/bin/env python3
"""Benchmark: T + T^H apply pairs per second on one MI355X.

Workload: 2D db4 tensor basis at J = 9 (512 x 512 coefficients), 1,048,576
Archimedean-spiral frequencies (64 arms x 16384, radius <= 256) with
Voronoi-area weights; FP32 applies (the metric form), weighted operator
A = W^{1/2} T as CGLS uses it, caller point order, inputs resident in HBM.

One step = one apply pair y = A x, z = A^H u through the C ABI.  Also
reported: FP64 apply pairs/s, per-kernel times (HIP events on the launch
stream), the roofline of the dominant kernel, the plan ("init") time,
wall time to relative normal residual 1e-6 for the plain FP64 and the
FP32-mixed CGLS, the batched solve of 64 uneven 2D problems (against the
same solves one after the other), the warm-start network (inference and
training throughput, conv roofline, and zero- against warm-start CGLS when
trained weights are present), and the FP64 CPU oracle timed on a bounded
sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu] [--no-batch] [--no-cnn]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes per launch of each kernel of the 2D tile path: every array
# the kernel must touch, read or written once (c = bytes per complex, r = bytes
# per real, pos = bytes per fixed-point coordinate).  nch = 2p boundary
# channels per dimension; tiles of 32 x 32 cells padded by W - 1.
def algorithmic_bytes(name, M, N, ng, nb, c, r, pos, W=8, TS=32):
    nbc = 2 * nb
    nt = (ng // TS) ** 2
    pw = TS + W - 1
    grid = ng * ng * c
    if name == "interp_bnd2d":      # coords, D_x, D_y, both boundary channel sets, boundary part out; side grids
        return M * (2 * pos + 2 * (nbc + 1) * c + c) + 2 * nbc * ng * c + nbc * nbc * c
    if name == "interp2d":          # coords, D_x, D_y, boundary part, sqrt(mu), perm, y out; grid once
        return M * (2 * pos + 2 * c + c + r + 4 + c) + grid
    if name == "adj_prep":          # u gathered through perm, sqrt(mu), sorted scaled input out
        return M * (c + 4 + r + c)
    if name == "spread2d":          # coords, scaled input, D_x, D_y, x-boundary channels; tile partials out
        return M * (2 * pos + c + 2 * c + nbc * c) + nt * (pw * pw + nbc * pw) * c
    if name == "boundary2d":        # x coordinate, scaled input, D_x, both boundary channel sets; partials out
        return M * (pos + c + c + 2 * nbc * c) + nt * (nbc * pw + nbc * nbc) * c
    if name == "merge_tiles":       # tile partials in; grid, side grids and corners out
        return nt * (pw * pw + 2 * nbc * pw + nbc * nbc) * c + grid + 2 * nbc * ng * c + nbc * nbc * c
    if name in ("fft_cols_T", "fft_cols_TH"):   # two passes, each reads and writes the grid
        return 4 * grid
    if name == "fft_rows_T":        # coefficients in, N transformed rows (interior and row sides) out
        return N * N * c + N * ng * c
    if name == "fft_rows_TH":
        return N * ng * c + N * N * c
    if name in ("fft_sidecols_T", "fft_sidecols_TH"):
        return 2 * nbc * ng * c
    return None


# Algorithmic bytes of one weighted apply pair (the method's stored-block
# formulation): per point coords, sqrt(mu), per-dimension scales, the 2dp
# boundary values and the in/out value; grid and FFT traffic ~ 13 N^2 c.
def pair_bytes(M, N, p, c, r, d=2):
    return 2 * (M * ((d + 1) * r + (d + 1 + 2 * d * p) * c) + 13 * N * N * c)


def oracle_baseline(pts, mu, J, p, sample, M):
    """FP64 oracle (dense per-dimension columns + BLAS) on a bounded sample:
    one weighted T and one T^H over `sample` points, scaled to pairs/s for M."""
    from oracle import basis
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(pts.shape[0], size=sample, replace=False))
    P = pts[idx]
    s = np.sqrt(mu[idx])
    N = 1 << J
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    u = rng.standard_normal(sample) + 1j * rng.standard_normal(sample)
    t0 = time.perf_counter()
    y = s * basis.apply_T_2d(P, J, p, X)
    Z = basis.apply_TH_2d(P, J, p, s * u)
    t = time.perf_counter() - t0
    assert np.isfinite(y).all() and np.isfinite(Z).all()
    cores = _blas_threads()
    return {"value": 1.0 / (t * M / sample), "unit": "pairs/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one weighted T and one T^H over {sample} of the {M} points (FP64, dense per-dimension "
                      f"columns + BLAS), {t:.2f} s, scaled linearly to all points"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def oracle_workloads(args, gpu_c1):
    """The oracle timed at the other workloads (FP64, all BLAS threads):
    one weighted apply pair at C1 (1D db2, J = 8, 1024 points k/2, whole),
    C2 (1D db4, J = 14, 65,536 jittered points; a seeded sample, scaled to all
    points) and C5 (2D db4, J = 8, 262,144 spiral points; a sample, scaled);
    the C1 least-squares solve (LAPACK lstsq on the dense T) on data the oracle
    forms itself; the C2 CGLS time extrapolated from the pair time and the
    GPU's iteration count (a full dense C2 CGLS takes tens of minutes)."""
    from oracle import basis, lsq
    from workloads import config_c1, config_c2, config_c5_pattern, complex_noise
    out = {}
    rng = np.random.default_rng(3)

    def pair_1d(xi, mu, J, p, x, u):
        s = np.sqrt(mu) if mu is not None else 1.0
        t0 = time.perf_counter()
        y = s * basis.apply_T_1d(xi, J, p, x, chunk=2048)
        z = basis.apply_TH_1d(xi, J, p, s * u, chunk=2048)
        t = time.perf_counter() - t0
        assert np.isfinite(y).all() and np.isfinite(z).all()
        return t

    c1 = config_c1()
    t = pair_1d(c1["xi"], None, c1["J"], c1["p"], c1["x0"], rng.standard_normal(c1["xi"].size) + 0j)
    T = basis.dense_T_1d(c1["xi"], c1["J"], c1["p"])
    y = T @ c1["x0"] + complex_noise(c1["xi"].size, c1["noise_sigma"], c1["noise_seed"])
    t0 = time.perf_counter()
    x_ls = lsq.lstsq_dense(T, y)
    t_ls = time.perf_counter() - t0
    out["c1"] = {"pairs_per_s": round(1.0 / t, 2), "sample": "all 1024 points", "lstsq_s": round(t_ls, 4)}
    if gpu_c1 is not None:
        out["c1"]["gpu_solution_vs_oracle_lstsq"] = float(np.linalg.norm(gpu_c1 - x_ls) / np.linalg.norm(x_ls))

    c2 = config_c2()
    n2 = min(args.cpu_sample // 8, c2["xi"].size)
    idx = np.sort(rng.choice(c2["xi"].size, n2, replace=False))
    t = pair_1d(c2["xi"][idx], c2["mu"][idx], c2["J"], c2["p"], c2["x0"], rng.standard_normal(n2) + 0j)
    t_full = t * c2["xi"].size / n2
    out["c2"] = {"pairs_per_s": round(1.0 / t_full, 5), "sample": f"{n2} of {c2['xi'].size} points, "
                 f"{t:.2f} s, scaled linearly", "pair_s": round(t_full, 2)}

    c5 = config_c5_pattern(with_weights=False)
    pts = c5["xi"]
    n5 = min(args.cpu_sample, pts.shape[0])
    idx = np.sort(rng.choice(pts.shape[0], n5, replace=False))
    N5 = 1 << c5["J"]
    X = rng.standard_normal((N5, N5)) + 1j * rng.standard_normal((N5, N5))
    t0 = time.perf_counter()
    yy = basis.apply_T_2d(pts[idx], c5["J"], c5["p"], X)
    zz = basis.apply_TH_2d(pts[idx], c5["J"], c5["p"], rng.standard_normal(n5) + 0j)
    t = time.perf_counter() - t0
    assert np.isfinite(yy).all() and np.isfinite(zz).all()
    out["c5"] = {"pairs_per_s": round(n5 / (t * pts.shape[0]), 4),
                 "sample": f"{n5} of {pts.shape[0]} points, {t:.2f} s, scaled linearly"}
    return out


def c1_solve(gs, torch, dev):
    """The 1D uniform workload (db2, J = 8, 1024 frequencies k/2, unit weights):
    the plan takes the exact uniform-node path (Sec. 3.2); y = T x0 by the
    library's FP64 apply plus 1e-8 complex noise; CGLS to 1e-10 (FP64)."""
    from workloads import config_c1, complex_noise
    c = config_c1()
    pl = gs.gs_plan(1, c["J"], c["p"], c["xi"], None, precision=gs.GS_F64)
    exact = pl.info()["exact_nodes"]
    x0 = torch.from_numpy(c["x0"]).to(dev)
    y = pl.apply_T(x0) + torch.from_numpy(complex_noise(c["xi"].size, c["noise_sigma"], c["noise_seed"])).to(dev)
    pl.solve(y, rel_tol=c["tol"], max_iter=2)                       # warm-up of the code path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = pl.solve(y, rel_tol=c["tol"], max_iter=500, check_every=10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pl.destroy()
    log(f"[bench] C1 solve (exact nodes: {exact}): {dt * 1e3:.2f} ms, {info['iterations']} iterations")
    return {"wall_s": round(dt, 5), "iterations": info["iterations"], "status": info["status"],
            "rel_residual": info["rel_residual"], "exact_nodes": bool(exact)}, x.cpu().numpy()


def batch_c4(gs, torch, dev, n_problems):
    """The batched workload: n_problems independent 2D problems (seeds
    4000 + b; J 6..9, db2/db4, jittered grid or spiral, M = 2..4 x 4^J),
    FP32-mixed plans, Voronoi weights (computed once, in a process pool,
    outside the timed region), y = T x0 (FP64 apply of the phantom).  Times
    the batched solve against the same solves run one after the other, and
    checks that each problem's result agrees."""
    from concurrent.futures import ProcessPoolExecutor
    from workloads import config_c4_problem
    t0 = time.time()
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        cfgs = list(ex.map(config_c4_problem, range(n_problems), ["voronoi"] * n_problems))
    plans = gs.gs_plan_batch([dict(dim=2, J=c["J"], p=c["p"], xi=c["xi"], mu=c["mu"], precision=gs.GS_F32_MIXED)
                              for c in cfgs])
    ys = []
    for c, pl in zip(cfgs, plans):
        y = torch.empty(pl.M, dtype=torch.complex128, device=dev)
        pl.apply_T(torch.from_numpy(c["x0"]).to(dev), y, f64=True)
        ys.append(y)
    torch.cuda.synchronize()
    total_m = sum(pl.M for pl in plans)
    log(f"[bench] batch: {n_problems} problems, {total_m} points, inputs and plans {time.time() - t0:.1f} s")
    kw = dict(rel_tol=1e-6, max_iter=1000, refine_fp64=True, max_restarts=3, check_every=10)
    gs.gs_solve_batch(plans, ys, rel_tol=1e-6, max_iter=2, check_every=1, n_streams=1)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lone_runs = [pl.solve(y, **kw) for pl, y in zip(plans, ys)]
    torch.cuda.synchronize()
    t_lone = time.perf_counter() - t0
    lone = [info for _, info in lone_runs]
    res = {}
    for ns in (1, 0):
        t0 = time.perf_counter()
        xs, infos = gs.gs_solve_batch(plans, ys, n_streams=ns, **kw)
        torch.cuda.synchronize()
        res[ns] = (time.perf_counter() - t0, infos, xs)
    t_batch, infos, xs = res[0]
    # equal to the lone solves: iteration counts, residuals and every solution entry bit for bit
    same = all(a["iterations"] == b["iterations"] and a["rel_residual"] == b["rel_residual"]
               for a, b in zip(lone, infos))
    same = same and all(torch.equal(xl, xb) for (xl, _), xb in zip(lone_runs, xs))
    classes = sorted({i["batch_class"] for i in infos})
    out = {"problems": n_problems, "points": int(total_m), "weights": "Voronoi areas",
           "geometry_classes": len(classes), "streams_chosen": infos[0]["batch_streams"],
           "wall_s": round(t_batch, 4), "wall_s_one_stream": round(res[1][0], 4),
           "lone_sequential_wall_s": round(t_lone, 4), "speedup_vs_lone": round(t_lone / t_batch, 3),
           "converged": sum(i["status"] == gs.GS_OK for i in infos),
           "iterations_max": max(i["iterations"] for i in infos),
           "iterations_sum": sum(i["iterations"] for i in infos),
           "max_rel_residual_fp64": max(i["rel_residual_fp64"] for i in infos),
           "equals_lone_solves": same}
    log(f"[bench] batch solve: {t_batch:.3f} s (one stream {res[1][0]:.3f} s), lone solves {t_lone:.3f} s, "
        f"{out['converged']}/{n_problems} converged, max iterations {out['iterations_max']}, "
        f"equal to lone: {same}")
    for pl in plans:
        pl.destroy()
    return out


CNN_WEIGHTS = os.path.join(ROOT, "paper_1607_04091_amd", "weights", "c5_cnn.npz")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "c3_spiral1M_traffic.json")
PAIR_SOURCES = ["paper_1607_04091_amd/csrc/nfft2d.hip", "paper_1607_04091_amd/csrc/nfft.hip",
                "paper_1607_04091_amd/csrc/fft.hpp", "paper_1607_04091_amd/csrc/common.hpp"]
CNN_SOURCES = ["paper_1607_04091_amd/csrc/cnn.hip"]
# bench kernel name -> substrings of the device kernel names (FP32 instances)
PMC_KERNELS = {
    "spread2d": ["adj_interior_kernel<float"], "boundary2d": ["adj_boundary_kernel<float"],
    "interp_bnd2d": ["interp_bnd_kernel<float"], "interp2d": ["interp_tile_kernel<float"],
    "adj_prep": ["adj_gather_kernel<float"], "merge_tiles": ["merge_kernel<float"],
    "cnn_conv32": ["conv32_kernel<0"],
}
COPY_MIB = 512


def _sources_sha1(files):
    import hashlib
    out = {}
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            out[f] = hashlib.sha1(fh.read()).hexdigest()
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when absent or when a kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("sources") != _sources_sha1(list(k.get("sources", {}))):
        return None
    return k["traffic_bytes"]


def pmc_run():
    """Workload for the counter passes: 3 FP32 apply pairs at the 1M-point
    spiral shape, 3 network forwards (batch 16, 256 x 256) and 3 plain copies
    of 512 MiB (an elementwise negation: reads and writes 512 MiB) that
    calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_1607_04091_amd import gs
    from workloads import spiral_2d, voronoi_weights_2d
    dev = torch.device("cuda:0")
    pts = spiral_2d(64, 16384, 256.0, 0.5)
    mu = voronoi_weights_2d(pts, "disk", 256.25, 0.4)
    plan = gs.gs_plan(2, 9, 4, pts, mu, precision=gs.GS_F32_MIXED)
    rng = np.random.default_rng(5)
    M, N = pts.shape[0], 512
    x = torch.from_numpy((rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)).to(dev)
    u = torch.from_numpy((rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(np.complex64)).to(dev)
    for _ in range(3):
        plan.apply_T(x, weighted=True)
        plan.apply_TH(u, weighted=True)
    net = gs.Cnn(256, 256, 16)
    net.set_weights(gs.cnn_he_init(7, last_scale=0.1))
    img = torch.zeros((16, 256, 256), dtype=torch.complex64, device=dev)
    for _ in range(3):
        net.forward(img)
    n = COPY_MIB * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    plan.destroy()
    net.destroy()
    print(json.dumps({"pmc_run": True}), flush=True)


def traffic_from(fetch_dir, write_dir, command):
    """Reads the counter CSVs of a FETCH_SIZE pass and a WRITE_SIZE pass,
    scales each by the copy kernel's reading of its known 512 MiB, and writes
    the per-launch HBM bytes of the kernels to profiles/ (JSON for bench.py,
    and a short table)."""
    import csv
    import glob

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        vals = {}
        for fn in files:
            with open(fn) as f:
                for row in csv.DictReader(f):
                    if row.get("Counter_Name") != counter:
                        continue
                    vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")

    def avg(vals, subs):
        tot, ok = 0.0, False
        for sub in subs:
            hits = [v for k, v in vals.items() if sub in k]
            if hits:
                ok = True
                tot += float(np.mean(hits[0]))
        return tot if ok else None

    copy_sub = ["neg_kernel", "neg"]
    fc = next((avg(fetch, [c]) for c in copy_sub if avg(fetch, [c]) is not None), None)
    wc = next((avg(write, [c]) for c in copy_sub if avg(write, [c]) is not None), None)
    if not fc or not wc:
        raise SystemExit("copy kernel not found in the counter output")
    kib = COPY_MIB * 1024.0
    cal = {"copy_mib": COPY_MIB, "fetch_kib": fc, "write_kib": wc, "fetch_scale": kib / fc, "write_scale": kib / wc}
    out = {"command": command, "calibration": cal, "kernels": {}}
    for name, subs in PMC_KERNELS.items():
        f, w = avg(fetch, subs), avg(write, subs)
        if f is None or w is None:
            continue
        fb, wb = f * 1024 * cal["fetch_scale"], w * 1024 * cal["write_scale"]
        src = CNN_SOURCES if name.startswith("cnn_") else PAIR_SOURCES
        out["kernels"][name] = {"fetch_kib": f, "write_kib": w, "fetch_bytes": fb, "write_bytes": wb,
                                "traffic_bytes": fb + wb, "sources": _sources_sha1(src)}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    lines = ["# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)", "",
             f"Command: `{command}`", "",
             f"Calibration: a {COPY_MIB} MiB elementwise copy reads {fc:.0f} KiB and writes {wc:.0f} KiB per "
             f"dispatch; scale factors {cal['fetch_scale']:.4f} (fetch), {cal['write_scale']:.4f} (write).", "",
             "| kernel | FETCH KiB | WRITE KiB | traffic MB (scaled) |", "|---|---|---|---|"]
    for name, k in out["kernels"].items():
        lines.append(f"| {name} | {k['fetch_kib']:.0f} | {k['write_kib']:.0f} | {k['traffic_bytes'] / 1e6:.1f} |")
    with open(TRAFFIC_JSON.replace(".json", ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(out["kernels"], indent=1))


def c2_solves(gs, torch, dev):
    """The 1D nonuniform workload (db4, J = 14, 65,536 jittered points,
    Voronoi lengths): wall time to relative normal residual 1e-8 for the FP64
    and the FP32-mixed solve, and the distance of the result from x0 (the data
    y = T x0 are consistent and T has full column rank, so the LS solution is
    x0).  y comes from the library's FP64 apply."""
    from workloads import config_c2
    c = config_c2()
    out = {}
    for name, prec in (("fp64", gs.GS_F64), ("fp32_mixed", gs.GS_F32_MIXED)):
        pl = gs.gs_plan(1, c["J"], c["p"], c["xi"], c["mu"], precision=prec)
        x0 = torch.from_numpy(c["x0"]).to(dev)
        y = pl.apply_T(x0, f64=prec == gs.GS_F32_MIXED)
        pl.solve(y, rel_tol=1e-8, max_iter=2)                      # warm-up of the code path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = pl.solve(y, rel_tol=1e-8, max_iter=1000, refine_fp64=True, max_restarts=3, check_every=10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(x - x0).item() / torch.linalg.vector_norm(x0).item())
        out[name] = {"wall_s": round(dt, 4), "iterations": info["iterations"], "status": info["status"],
                     "rel_residual": info["rel_residual"], "rel_residual_fp64": info["rel_residual_fp64"],
                     "rel_error_vs_x0": err}
        log(f"[bench] C2 solve {name}: {dt * 1e3:.1f} ms, {info['iterations']} iterations, status {info['status']}, "
            f"|x - x0|/|x0| {err:.2e}")
        pl.destroy()
    return out


def cnn_bench(gs, torch, dev, batch, steps, n_eval):
    """The learned warm start on its workload (db4, J = 8, 256 x 256, 64 x 4096
    spiral points, radius 128, Voronoi weights): network throughput for
    inference and training on batches of 256 x 256 images, per-kernel times,
    the roofline of the hidden-layer convolution, and -- with trained weights
    present -- zero-start against warm-start CGLS to 1e-6 on held-out
    phantoms (seeds 70000...)."""
    from paper_1607_04091_amd import warmstart as ws
    H = W = 256
    net = gs.Cnn(H, W, batch)
    trained = os.path.exists(CNN_WEIGHTS)
    if trained:
        net.load(CNN_WEIGHTS)
    else:
        net.set_weights(gs.cnn_he_init(7, last_scale=0.1))
    rng = np.random.default_rng(9)
    x = torch.from_numpy((rng.standard_normal((batch, H, W)) + 1j * rng.standard_normal((batch, H, W)))
                         .astype(np.complex64)).to(dev)
    t = x * 0.5
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def timed(fn, n, warm=3):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    ms_inf = timed(lambda: net.forward(x, out, stream=stream), steps)

    def train_step():
        net.forward(x, train=True, stream=stream)
        net.backward(t, stream=stream, want_loss=False)
        net.step(1e-6, stream=stream)

    ms_train = timed(train_step, max(3, steps // 2))
    gs.gs_profile_enable(True)
    nprof = 5
    for _ in range(nprof):
        train_step()
    torch.cuda.synchronize()
    prof = gs.gs_profile_read()
    gs.gs_profile_enable(False)
    if trained:
        net.load(CNN_WEIGHTS)                   # undo the timing steps
    kern = {k: {"launches": n, "avg_us": 1000.0 * tt / n} for k, (n, tt) in prof.items() if k.startswith("cnn_")}
    flop_img = 2 * H * W * 9 * (2 * 32 + 4 * 32 * 32 + 32 * 2)
    conv = kern.get("cnn_conv32")
    roof = None
    if conv:
        byts = batch * H * W * 64 * 2           # read and write one bf16 activation tensor per launch
        ach = byts / (conv["avg_us"] * 1e-6) / 1e9
        fl = batch * 2 * H * W * 9 * 32 * 32 / (conv["avg_us"] * 1e-6) / 1e12
        roof = {"kernel": "cnn_conv32", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic("cnn_conv32"),
                "tflops_bf16": round(fl, 1),
                "mfma_frac_bf16": round(fl / 2500.0, 4), "avg_launch_us": round(conv["avg_us"], 2),
                "algorithmic_bytes_per_launch": int(byts)}
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["avg_us"] * kv[1]["launches"]):
        log(f"[bench]   {k:20s} {v['launches']:5d} launches  avg {v['avg_us']:9.2f} us")
    res = {"batch": batch, "image": [H, W], "inference_ms": round(ms_inf, 3),
           "inference_images_per_s": round(batch * 1000 / ms_inf, 1),
           "inference_tflops": round(batch * flop_img / (ms_inf * 1e-3) / 1e12, 2),
           "train_step_ms": round(ms_train, 3), "train_images_per_s": round(batch * 1000 / ms_train, 1),
           "kernels_us": {k: round(v["avg_us"], 2) for k, v in kern.items()}, "conv_roofline": roof,
           "trained_weights": trained}
    log(f"[bench] cnn: inference {ms_inf:.3f} ms / {batch} images, training step {ms_train:.3f} ms")
    if trained and n_eval > 0:
        plans, c = ws.c5_plans(1)
        rows = ws.evaluate(plans[0], net, np.arange(70000, 70000 + n_eval), c["J"])
        res["warm_vs_zero"] = ws.summarize(rows)
        log(f"[bench] warm start: {res['warm_vs_zero']}")
        plans[0].destroy()
    net.destroy()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--no-cnn", action="store_true")
    ap.add_argument("--warm-eval", type=int, default=100)
    ap.add_argument("--cpu-sample", type=int, default=32768)
    ap.add_argument("--arms", type=int, default=64)
    ap.add_argument("--per-arm", type=int, default=16384)
    ap.add_argument("--pmc-run", action="store_true", help="only the short workload for counter passes")
    ap.add_argument("--traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="turn two counter passes into profiles/c3_spiral1M_traffic.{json,md} (no GPU)")
    args = ap.parse_args()
    if args.traffic:
        traffic_from(*args.traffic)
        return
    if args.pmc_run:
        pmc_run()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the point-sharded design "
              "is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1607_04091_amd import gs
    from workloads import spiral_2d, voronoi_weights_2d, ellipse_phantom_params, phantom_cell_averages, \
        relative_noise

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    dev = torch.device("cuda:0")
    J, p = 9, 4
    N = 1 << J
    r_max = 256.0
    t0 = time.time()
    pts = spiral_2d(args.arms, args.per_arm, r_max, 0.5)
    mu = voronoi_weights_2d(pts, "disk", r_max + 0.25, 0.4)
    M = pts.shape[0]
    x0 = phantom_cell_averages(ellipse_phantom_params(301), J).astype(np.complex128)
    log(f"[bench] inputs: M={M} spiral points, Voronoi weights ({time.time() - t0:.1f} s)")

    # init as the paper times it (the first run excluded): the first plan of the
    # process also loads the code objects and builds the host filter tables
    t0 = time.perf_counter()
    plan = gs.gs_plan(2, J, p, pts, mu, precision=gs.GS_F32_MIXED)
    torch.cuda.synchronize()
    t_init_first = time.perf_counter() - t0
    plan.destroy()
    t0 = time.perf_counter()
    plan = gs.gs_plan(2, J, p, pts, mu, precision=gs.GS_F32_MIXED)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    log(f"[bench] plan (init, FP32+FP64 data): {t_init:.3f} s (first in the process {t_init_first:.3f} s), "
        f"device bytes {plan.info()['device_bytes'] / 2**20:.0f} MiB")

    rng = np.random.default_rng(5)
    xs = torch.from_numpy(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).to(dev)
    us = torch.from_numpy(rng.standard_normal(M) + 1j * rng.standard_normal(M)).to(dev)
    x32, u32 = xs.to(torch.complex64), us.to(torch.complex64)
    y32 = torch.empty(M, dtype=torch.complex64, device=dev)
    z32 = torch.empty((N, N), dtype=torch.complex64, device=dev)
    y64 = torch.empty(M, dtype=torch.complex128, device=dev)
    z64 = torch.empty((N, N), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def pair32():
        plan.apply_T(x32, y32, weighted=True, stream=stream)
        plan.apply_TH(u32, z32, weighted=True, stream=stream)

    def pair64():
        plan.apply_T(xs, y64, weighted=True, f64=True, stream=stream)
        plan.apply_TH(us, z64, weighted=True, f64=True, stream=stream)

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms32 = timed(pair32, args.steps, args.warmup)
    log(f"[bench] FP32 pair: {ms32:.3f} ms -> {1000 / ms32:.1f} pairs/s")
    ms64 = timed(pair64, max(3, args.steps // 5), 2)
    log(f"[bench] FP64 pair: {ms64:.3f} ms -> {1000 / ms64:.1f} pairs/s")
    assert torch.isfinite(torch.view_as_real(y32)).all() and torch.isfinite(torch.view_as_real(z32)).all()

    # per-kernel times of the FP32 pair, HIP events on the launch stream
    gs.gs_profile_enable(True)
    nprof = max(5, min(args.steps, 20))
    for _ in range(nprof):
        pair32()
    torch.cuda.synchronize()
    prof = gs.gs_profile_read()
    gs.gs_profile_enable(False)
    kernels = {k: {"launches": n, "avg_us": 1000.0 * t / n} for k, (n, t) in prof.items()}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"] / nprof)
    for k, v in kernels.items():
        ab = algorithmic_bytes(k, M, N, 2 * N, p, 8, 4, 4)
        if ab is not None:
            v["gbs"] = ab / (v["avg_us"] * 1e-6) / 1e9
    ab = algorithmic_bytes(dom, M, N, 2 * N, p, 8, 4, 4)
    roof = None
    if ab is not None:
        ach = ab / (kernels[dom]["avg_us"] * 1e-6) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                "algorithmic_bytes_per_launch": int(ab), "avg_launch_us": round(kernels[dom]["avg_us"], 2)}
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_us"] * kv[1]["launches"]):
        log(f"[bench]   {k:20s} {v['launches']:5d} launches  avg {v['avg_us']:9.2f} us"
            + (f"  {v['gbs']:7.0f} GB/s algorithmic" if "gbs" in v else ""))
    pb = pair_bytes(M, N, p, 8, 4)
    pair_roof = {"algorithmic_bytes": int(pb), "achieved_gbs": round(pb / (ms32 * 1e-3) / 1e9, 1),
                 "frac": round(pb / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "ceiling_pairs_per_s": round(HBM_PEAK_GBS * 1e9 / pb, 1)}

    solve = {}
    c1_x = None
    if not args.no_solve:
        x0d = torch.from_numpy(x0).to(dev)
        yclean = torch.empty(M, dtype=torch.complex128, device=dev)
        plan.apply_T(x0d, yclean, f64=True, stream=stream)
        torch.cuda.synchronize()
        ynp = yclean.cpu().numpy()
        y = torch.from_numpy(ynp + relative_noise(ynp, 1e-4, 302)).to(dev)
        sols = {}
        for name, prec in (("fp32_mixed", gs.GS_F32_MIXED), ("plain_fp64", gs.GS_F64)):
            pl = plan if prec == gs.GS_F32_MIXED else gs.gs_plan(2, J, p, pts, mu, precision=prec)
            xsol = torch.zeros((N, N), dtype=torch.complex128, device=dev)
            pl.solve(y, xsol, rel_tol=1e-6, max_iter=2, check_every=1)     # warm-up of the code path
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xsol, info = pl.solve(y, xsol, rel_tol=1e-6, max_iter=1000, refine_fp64=True, max_restarts=3,
                                  check_every=10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            solve[name] = {"wall_s": round(dt, 4), "iterations": info["iterations"],
                           "restarts": info["restarts"], "status": info["status"],
                           "rel_residual": info["rel_residual"], "rel_residual_fp64": info["rel_residual_fp64"]}
            log(f"[bench] solve {name}: {dt:.3f} s, {info['iterations']} iterations, status {info['status']}, "
                f"rr {info['rel_residual']:.2e}, rr64 {info['rel_residual_fp64']:.2e}")
            sols[name] = xsol
            if pl is not plan:
                pl.destroy()
        # the mixed-form result against the plain FP64 solve of the same problem
        d = torch.linalg.vector_norm(sols["fp32_mixed"] - sols["plain_fp64"]).item()
        solve["fp32_mixed"]["rel_diff_vs_plain_fp64"] = d / torch.linalg.vector_norm(sols["plain_fp64"]).item()
        log(f"[bench] mixed vs plain FP64 solution: {solve['fp32_mixed']['rel_diff_vs_plain_fp64']:.2e}")
        solve["warm_start"] = None
        solve["c1_1d"], c1_x = c1_solve(gs, torch, dev)
        solve["c2_1d"] = c2_solves(gs, torch, dev)
        if not args.no_batch:
            solve["batched_c4"] = batch_c4(gs, torch, dev, args.batch_problems)

    cnn = None
    if not args.no_cnn:
        cnn = cnn_bench(gs, torch, dev, 16, 20, 0 if args.no_solve else args.warm_eval)
        if "warm_vs_zero" in cnn:
            solve["warm_start"] = cnn["warm_vs_zero"]

    cpu = None
    if not args.no_cpu:
        cpu = oracle_baseline(pts, mu, J, p, min(args.cpu_sample, M), M)
        log(f"[bench] oracle: {cpu['value']:.3e} pairs/s on {cpu['cores']} threads")
        cpu["cpu_model"] = _cpu_model()
        cpu["host_cpus"] = os.cpu_count()
        cpu["workloads"] = oracle_workloads(args, c1_x)
        c2_it = (solve.get("c2_1d") or {}).get("fp64", {}).get("iterations")
        if c2_it:
            cpu["workloads"]["c2"]["cgls_s_extrapolated"] = round(cpu["workloads"]["c2"]["pair_s"] * c2_it, 1)
            cpu["workloads"]["c2"]["cgls_iterations_assumed"] = c2_it
        log(f"[bench] oracle workloads: {json.dumps(cpu['workloads'])}")

    line = {
        "metric": "T+T^H apply pairs/s (2D 512², 1M pts); time-to-rel-res 1e-6 plain vs warm-start",
        "value": round(1000.0 / ms32, 2),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D db4 J=9 (512x512 coefficients), {M} Archimedean-spiral frequencies "
                               f"({args.arms} arms, radius <= 256), Voronoi-area weights, weighted T and T^H, FP32",
                   "points": M, "coefficients": N * N, "parallelism": "single GPU"},
        "fp64_pairs_per_s": round(1000.0 / ms64, 2),
        "init_s": round(t_init, 3), "init_first_in_process_s": round(t_init_first, 3),
        "kernels_us": {k: round(v["avg_us"], 2) for k, v in kernels.items()},
        "roofline": roof,
        "pair_roofline": pair_roof,
        "solve": solve,
        "cnn": cnn,
        "cpu_baseline": cpu,
    }
    plan.destroy()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
