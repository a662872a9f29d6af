"""Learned CGLS warm start for 2D generalized-sampling problems (this
library's addition; the paper starts CGLS from zero).

* ``adjoint_image``  -- A^H b = T^H W y, the network's input (one apply).
* ``generate``       -- training pairs made by the method itself: phantom
                        coefficients x0, data y = T x0 (+ relative noise),
                        input A^H b and target = the CGLS solution, solved
                        with the batched solver over several plans of the
                        same sampling pattern.
* ``train``          -- Adam on the library's CNN kernels, cosine learning
                        rate, random mini-batches.
* ``warm_solve``     -- x0 = CNN(A^H b), then gs_solve with the guarded warm
                        start: if x0's normal residual is not below that of
                        x0 = 0, the solve starts from zero instead.

Command line (one GPU):
  python -m paper_1607_04091_amd.warmstart train --out c5_cnn.npz \\
      [--train 20000] [--test 100] [--epochs 4] [--batch 16]
trains on the 256 x 256 spiral workload (db4, J = 8, 64 arms x 4096 points,
radius 128, Voronoi weights) and reports zero-start against warm-start
CGLS on held-out phantoms.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import gs


def adjoint_image(plan, y, out=None, stream=None):
    """A^H b = T^H W y as a complex128 N x N tensor (FP64 apply)."""
    if plan.precision == gs.GS_F32:
        raise ValueError("the warm start needs a plan with FP64 data (GS_F64 or GS_F32_MIXED)")
    return plan.apply_TH(y, out, weighted="full", f64=plan.precision == gs.GS_F32_MIXED, stream=stream)


def _noisy_data(plan, x0, noise_rel, seed):
    """y = T x0 (FP64 apply) plus complex Gaussian noise of relative size
    noise_rel (seeded torch generator on the device)."""
    import torch
    y = torch.empty(plan.M, dtype=torch.complex128, device=x0.device)
    plan.apply_T(x0.to(torch.complex128).contiguous(), y, f64=plan.precision == gs.GS_F32_MIXED)
    if noise_rel > 0:
        g = torch.Generator(device=x0.device)
        g.manual_seed(int(seed))
        n = torch.randn((plan.M, 2), dtype=torch.float64, device=x0.device, generator=g)
        sigma = noise_rel * torch.linalg.vector_norm(y).item() / math.sqrt(2 * plan.M)
        y += sigma * torch.view_as_complex(n)
    return y


def generate(plans, seeds, J, noise_rel=1e-4, tol=1e-6, max_iter=1000, log=None, seconds=None):
    """Training pairs for phantoms with the given seeds.  plans: several
    plans of one sampling pattern (FP32-mixed), solved together.  Returns
    (inputs, targets) as complex64 (n, N, N) device tensors and the CGLS
    iteration counts.  With `seconds`, stops early (after a whole chunk) once
    that much time has passed and returns the pairs made so far."""
    import torch
    from workloads import ellipse_phantom_params, phantom_cell_averages_torch
    dev = torch.device("cuda")
    N = 1 << J
    n, K = len(seeds), len(plans)
    inputs = torch.empty((n, N, N), dtype=torch.complex64, device=dev)
    targets = torch.empty((n, N, N), dtype=torch.complex64, device=dev)
    iters = []
    t0 = time.time()
    done = 0
    for start in range(0, n, K):
        if seconds is not None and time.time() - t0 > seconds:
            break
        chunk = seeds[start:start + K]
        x0s = phantom_cell_averages_torch([ellipse_phantom_params(int(s)) for s in chunk], J, dev)
        ys = []
        for k, s in enumerate(chunk):
            y = _noisy_data(plans[k], x0s[k], noise_rel, 1_000_000 + int(s))
            ys.append(y)
            inputs[start + k] = adjoint_image(plans[k], y).to(torch.complex64)
        xs, infos = gs.gs_solve_batch(plans[:len(chunk)], ys, rel_tol=tol, max_iter=max_iter, refine_fp64=True,
                                      max_restarts=3, check_every=10)
        for k in range(len(chunk)):
            targets[start + k] = xs[k].to(torch.complex64)
            iters.append(infos[k]["iterations"])
        done = start + len(chunk)
        if log and (start // K) % max(1, (n // K) // 10) == 0:
            log(f"[warmstart] data {start + len(chunk)}/{n} ({time.time() - t0:.1f} s)")
    return inputs[:done], targets[:done], iters


def fit_input_scale(inputs, targets, count=64):
    """Fixed input scale: the median of ||target|| / ||input|| over a sample."""
    import torch
    k = min(count, inputs.shape[0])
    a = torch.linalg.vector_norm(inputs[:k].reshape(k, -1), dim=1)
    b = torch.linalg.vector_norm(targets[:k].reshape(k, -1), dim=1)
    return float(torch.median(b / a).item())


def train(net, inputs, targets, epochs=4, batch=16, lr_max=1e-3, lr_min=1e-5, seed=0, log=None, log_every=200):
    """Adam over random mini-batches, cosine learning rate from lr_max to
    lr_min.  Returns the logged (step, loss) pairs."""
    import torch
    n = inputs.shape[0]
    if n < batch:
        raise ValueError("fewer training pairs than one batch")
    spe = n // batch
    total = epochs * spe
    rng = np.random.default_rng(seed)
    xb = torch.empty((batch,) + tuple(inputs.shape[1:]), dtype=inputs.dtype, device=inputs.device)
    tb = torch.empty_like(xb)
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(inputs.device)
        for i in range(spe):
            idx = perm[i * batch:(i + 1) * batch]
            torch.index_select(inputs, 0, idx, out=xb)
            torch.index_select(targets, 0, idx, out=tb)
            net.forward(xb, train=True)
            want = (step % log_every == 0) or step == total - 1
            loss = net.backward(tb, want_loss=want)
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * step / max(1, total - 1)))
            net.step(lr)
            if want:
                hist.append((step, loss))
                if log:
                    log(f"[warmstart] step {step}/{total} epoch {ep} loss {loss:.4e} lr {lr:.2e} "
                        f"({time.time() - t0:.1f} s)")
            step += 1
    return hist


def warm_solve(plan, y, net, rel_tol=1e-6, max_iter=1000, check_every=10, stream=None):
    """x0 = net(A^H b), then CGLS with the guarded warm start."""
    import torch
    img = adjoint_image(plan, y, stream=stream)
    x0 = net.forward(img, out_dtype=torch.complex128, stream=stream)
    return plan.solve(y, x0, rel_tol=rel_tol, max_iter=max_iter, warm_start="guarded", refine_fp64=True,
                      max_restarts=3, check_every=check_every, stream=stream)


def evaluate(plan, net, seeds, J, noise_rel=1e-4, tol=1e-6, log=None):
    """Zero-start against warm-start CGLS on phantoms with the given seeds.
    Wall times include, for the warm start, A^H b and the network."""
    import torch
    from workloads import ellipse_phantom_params, phantom_cell_averages_torch
    dev = torch.device("cuda")
    rows = []
    N = 1 << J
    # warm-up of both code paths
    x0s = phantom_cell_averages_torch([ellipse_phantom_params(int(seeds[0]))], J, dev)
    y = _noisy_data(plan, x0s[0], noise_rel, 1_000_000 + int(seeds[0]))
    plan.solve(y, rel_tol=tol, max_iter=3)
    warm_solve(plan, y, net, rel_tol=tol, max_iter=3)
    for s in seeds:
        x0s = phantom_cell_averages_torch([ellipse_phantom_params(int(s))], J, dev)
        y = _noisy_data(plan, x0s[0], noise_rel, 1_000_000 + int(s))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xz, iz = plan.solve(y, torch.zeros((N, N), dtype=torch.complex128, device=dev), rel_tol=tol, max_iter=1000,
                            refine_fp64=True, max_restarts=3, check_every=10)
        torch.cuda.synchronize()
        tz = time.perf_counter() - t0
        t0 = time.perf_counter()
        xw, iw = warm_solve(plan, y, net, rel_tol=tol)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        rows.append({"seed": int(s), "zero_iters": iz["iterations"], "zero_s": tz, "zero_status": iz["status"],
                     "zero_rr64": iz["rel_residual_fp64"], "warm_iters": iw["iterations"], "warm_s": tw,
                     "warm_status": iw["status"], "warm_rr64": iw["rel_residual_fp64"],
                     "warm_used": iw["warm_start_used"]})
        if log:
            r = rows[-1]
            log(f"[warmstart] eval seed {s}: zero {r['zero_iters']} it {tz * 1e3:.1f} ms | warm {r['warm_iters']} it "
                f"{tw * 1e3:.1f} ms used={r['warm_used']}")
    return rows


def summarize(rows):
    z = np.array([r["zero_iters"] for r in rows], float)
    w = np.array([r["warm_iters"] for r in rows], float)
    return {"problems": len(rows), "zero_iters_mean": float(z.mean()), "warm_iters_mean": float(w.mean()),
            "zero_s_mean": float(np.mean([r["zero_s"] for r in rows])),
            "warm_s_mean": float(np.mean([r["warm_s"] for r in rows])),
            "warm_used": int(sum(r["warm_used"] for r in rows)),
            "all_converged": bool(all(r["zero_status"] == gs.GS_OK and r["warm_status"] == gs.GS_OK for r in rows)),
            "max_rr64_zero": float(max(r["zero_rr64"] for r in rows)),
            "max_rr64_warm": float(max(r["warm_rr64"] for r in rows))}


def c5_plans(count, precision=None):
    """Plans of the warm-start workload: db4, J = 8, 64 x 4096 spiral points,
    radius 128, Voronoi weights."""
    from workloads import config_c5_pattern
    c = config_c5_pattern()
    prec = gs.GS_F32_MIXED if precision is None else precision
    return [gs.gs_plan(2, c["J"], c["p"], c["xi"], c["mu"], precision=prec) for _ in range(count)], c


def _log(msg):
    print(msg, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1607_04091_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--train", type=int, default=20000)
    t.add_argument("--test", type=int, default=100)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--plans", type=int, default=8)
    t.add_argument("--data-seconds", type=float, default=None,
                   help="stop making training pairs after this many seconds")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        _log("no GPU")
        return 1
    t0 = time.time()
    plans, c = c5_plans(args.plans)
    J = c["J"]
    N = 1 << J
    _log(f"[warmstart] {len(plans)} plans, M={plans[0].M}, J={J} ({time.time() - t0:.1f} s)")
    tr_seeds = np.arange(50000, 50000 + args.train)
    inputs, targets, iters = generate(plans, tr_seeds, J, log=_log, seconds=args.data_seconds)
    t_data = time.time() - t0
    _log(f"[warmstart] training data: {inputs.shape[0]} pairs, mean CGLS iterations {np.mean(iters):.1f} "
         f"({t_data:.1f} s)")
    net = gs.Cnn(N, N, args.batch)
    net.set_weights(gs.cnn_he_init(7, last_scale=0.1))
    net.input_scale = fit_input_scale(inputs, targets)
    _log(f"[warmstart] input scale {net.input_scale:.4e}")
    t1 = time.time()
    hist = train(net, inputs, targets, epochs=args.epochs, batch=args.batch, lr_max=args.lr, log=_log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    net.save(args.out)
    del inputs, targets
    for pl in plans[1:]:
        pl.destroy()
    rows = evaluate(plans[0], net, np.arange(70000, 70000 + args.test), J, log=_log)
    summ = summarize(rows)
    meta = {"train_pairs": int(len(iters)), "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "data_s": round(t_data, 1), "train_s": round(t_train, 1), "input_scale": net.input_scale,
            "loss_history": hist, "target_iters_mean": float(np.mean(iters)), "eval": summ}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    _log("[warmstart] " + json.dumps(summ))
    plans[0].destroy()
    return 0


if __name__ == "__main__":
    sys.exit(main())
