#!/usr/bin/env python
"""Throughput of the rank-truncated PCG solve on one MI355X.

A step is one complete solve (Algorithm 1 of the paper with the entry and
exit transforms and the Tucker-to-canonical output) of the control equation
(beta A^-alpha + (gamma/beta) A^alpha) u = y for one design function, with the
plan (eigenpairs, separable operator and preconditioner) built beforehand and
the inputs resident in HBM.  Default workload: n = 1024 per mode,
a_l(x) = 1 + 0.9 sin(4 pi x + phi_l), rank-10 Gaussian-bump design, alpha = 0.5,
beta = 1e-4, gamma = 1, eps = 1e-6, FP64.

Prints one JSON line (rank 0) with the solves/sec, the roofline of the
dominant kernel (the FP64 matrix-core GEMM, timed with HIP events on its
stream inside the timed region), the CPU oracle timed on a bounded sample on
this host, and the oracle error of the last solve on sampled slabs.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rank-truncated PCG solves/sec at n=1024, ε=1e-6: mixed/batched vs FP64"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads as wl
    if name == "sine1024":
        return wl.workload_sine(n=1024, seed=3), "sine_n1024_rank10"
    if name == "quad256":
        return wl.workload_quadratic(n=256, alpha=0.5), "quadratic_n256_rank5"
    if name == "small":
        return wl.workload_small(), "small_n32_rank1"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(prob, sample_slabs=8):
    """The oracle's exact solve, timed on a bounded sample: full setup (three
    LAPACK tridiagonal eigensolves and the entry transform), then the divide
    and the mode-2/3 products for `sample_slabs` of the n mode-1 slabs and the
    mode-1 product for the same share of columns; extrapolated to all n
    slabs."""
    import numpy as np
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n = prob.n
    t0 = time.perf_counter()
    sp = osolve.Spectral(prob)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    blk = osolve.solve_eig_block(sp, 0, sample_slabs)
    blk = np.tensordot(blk, sp.V[1], axes=(1, 1))          # (b, k, j) <- mode 2
    blk = np.tensordot(blk, sp.V[2], axes=(1, 1))          # (b, j, k) <- mode 3
    t_slabs = time.perf_counter() - t0
    cols = blk.reshape(sample_slabs, -1)
    W = np.ascontiguousarray(np.random.default_rng(0).standard_normal((n, sample_slabs)))
    t0 = time.perf_counter()
    _ = W @ cols                                           # mode-1 product share
    t_mode1 = time.perf_counter() - t0
    scale = n / sample_slabs
    t_total = t_setup + scale * (t_slabs + t_mode1)
    return {
        "value": 1.0 / t_total, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
        "sample": (f"oracle exact solve at n={n}: setup timed in full ({t_setup:.2f}s), divide + "
                   f"mode-2/3 products timed on {sample_slabs} of {n} mode-1 slabs and the mode-1 "
                   f"product on the same share of columns, extrapolated x{scale:.0f}; "
                   f"estimated {t_total:.1f}s per solve"),
    }


def measure_batched(args, api, torch, dev):
    """Many independent solves in one fc_solve_batched call (concurrent
    streams): `batch` problems of the sine family at n = 1024 with seeds
    100.. (or the uneven-size family), plans built beforehand."""
    import numpy as np
    import threading
    import workloads as wl
    from oracle import solve as osolve
    if args.batch_workload == "mixed":
        probs = wl.workload_batched(count=args.batch)
    else:
        probs = wl.workload_batched_uniform(count=args.batch, n=1024)
    log(f"[bench] batched: {len(probs)} problems ({args.batch_workload}); building plans ...")
    t0 = time.perf_counter()
    plans = [None] * len(probs)

    def build(i):
        p = probs[i]
        plans[i] = api.Plan(p.n, p.a, p.alpha, p.beta, p.gamma, p.eps)

    idx = list(range(len(probs)))
    th = []
    for t in range(8):
        th.append(threading.Thread(target=lambda t=t: [build(i) for i in idx[t::8]]))
        th[-1].start()
    for x in th:
        x.join()
    setup_s = time.perf_counter() - t0
    log(f"[bench] batched setup {setup_s:.1f}s")
    inputs = [(torch.from_numpy(np.asarray(p.w)).to(dev),
               [api.to_device_colmajor(y, dev) for y in p.Y]) for p in probs]
    cap = 1024
    outs = [(torch.empty(cap, dtype=torch.float64, device=dev),
             [torch.empty((cap, p.n), dtype=torch.float64, device=dev).t() for _ in range(3)])
            for p in probs]
    res = api.solve_batched(plans, inputs, cap_u=cap, outs=outs)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.batch_steps):
        res = api.solve_batched(plans, inputs, cap_u=cap, outs=outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rate = args.batch_steps * len(probs) / el
    log(f"[bench] batched: {args.batch_steps} x {len(probs)} solves in {el:.2f}s -> {rate:.2f} solves/s")
    checks = []
    if not args.no_check:
        rng = np.random.default_rng(1)
        for i in [0, len(probs) - 1]:
            p = probs[i]
            w_u, U, info, st = res[i]
            slabs = sorted(set(list(range(8)) + list(rng.choice(p.n, size=8, replace=False))))
            rep = osolve.rel_error(p, w_u.cpu().numpy(), [u.cpu().numpy() for u in U], slabs=slabs)
            checks.append({"problem": i, "n": p.n, "rel_l2_sampled": rep["rel_l2"],
                           "slabs": rep["slabs"], "iterations": info["iterations"],
                           "pass": bool(rep["rel_l2"] <= 10 * p.eps)})
        log(f"[bench] batched checks {checks}")
    for p in plans:
        p.close()
    iters = [r[2]["iterations"] for r in res]
    return {"workload": args.batch_workload, "problems": len(probs), "steps": args.batch_steps,
            "solves_per_s": rate, "s_per_batch": el / args.batch_steps, "setup_s": setup_s,
            "streams": int(os.environ.get("FC_BATCH_STREAMS", "8")),
            "iterations_min_max": [min(iters), max(iters)], "checks": checks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sine1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--check-slabs", type=int, default=24)
    ap.add_argument("--batch", type=int, default=64,
                    help="problems in the batched measurement (0 disables it)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--batch-workload", default="sine1024x64")
    ap.add_argument("--mixed-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method runs on a single device; see the multi-GPU design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2006_09314_amd import api
    from paper_2006_09314_amd._lib import check, lib

    prob, wname = make_workload(args.workload)
    log(f"[bench] workload {wname}: n={prob.n} rank_y={prob.rank} alpha={prob.alpha} "
        f"beta={prob.beta} eps={prob.eps}")
    torch.cuda.init()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = api.Plan(prob.n, prob.a, prob.alpha, prob.beta, prob.gamma, prob.eps)
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f}s")
    w = torch.from_numpy(np.asarray(prob.w)).to(dev)
    Y = [api.to_device_colmajor(y, dev) for y in prob.Y]
    cap = 8192
    out = (torch.empty(cap, dtype=torch.float64, device=dev),
           [torch.empty((cap, prob.n), dtype=torch.float64, device=dev).t() for _ in range(3)])
    info = None
    for i in range(args.warmup):
        res = plan.solve(w, Y, cap_u=cap, out=out)
        info = res[2]
        log(f"[bench] warmup {i}: {info}")
    torch.cuda.synchronize()
    check(lib().fc_profile_gemm(1), "fc_profile_gemm")
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = plan.solve(w, Y, cap_u=cap, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check(lib().fc_profile_gemm(0), "fc_profile_gemm")
    info = res[2]
    launches, ms, flops, byts = C.c_long(), C.c_double(), C.c_double(), C.c_double()
    check(lib().fc_profile_gemm_read(C.byref(launches), C.byref(ms), C.byref(flops), C.byref(byts)),
          "fc_profile_gemm_read")
    elapsed = t1 - t0
    value = args.steps / elapsed
    log(f"[bench] timed {args.steps} solves in {elapsed:.3f}s -> {value:.2f} solves/s")

    per_launch_s = (ms.value / 1e3) / max(launches.value, 1)
    fl_launch = flops.value / max(launches.value, 1)
    by_launch = byts.value / max(launches.value, 1)
    ai = flops.value / max(byts.value, 1.0)
    if ai >= PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        achieved = fl_launch / per_launch_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
    else:
        achieved = by_launch / per_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof.update({"kernel": "gemm_kernel (FP64 MFMA 16x16x4)", "launches_per_step":
                 launches.value / args.steps, "avg_launch_us": per_launch_s * 1e6,
                 "flops_per_launch": fl_launch, "bytes_per_launch": by_launch,
                 "gemm_share_of_step": (ms.value / 1e3) / elapsed})

    mixed = None
    if args.mixed_steps > 0:
        mplan = api.Plan(prob.n, prob.a, prob.alpha, prob.beta, prob.gamma, prob.eps, precision=1)
        res_m = mplan.solve(w, Y, cap_u=cap, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.mixed_steps):
            res_m = mplan.solve(w, Y, cap_u=cap, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mixed = {"solves_per_s": args.mixed_steps / el, "ms_per_solve": 1e3 * el / args.mixed_steps,
                 "info": res_m[2]}
        if not args.no_check:
            from oracle import solve as osolve
            rng = np.random.default_rng(2)
            slabs = sorted(set(list(range(12)) + list(rng.choice(prob.n, size=8, replace=False))))
            rep = osolve.rel_error(prob, res_m[0].cpu().numpy(), [u.cpu().numpy() for u in res_m[1]],
                                   slabs=slabs)
            mixed["rel_l2_sampled"] = rep["rel_l2"]
            mixed["pass"] = bool(rep["rel_l2"] <= 10 * prob.eps)
        log(f"[bench] mixed FP32/FP64-refinement: {mixed}")
        mplan.close()

    batched = None
    if args.batch > 0:
        batched = measure_batched(args, api, torch, dev)

    parity = None
    if not args.no_check:
        from oracle import solve as osolve
        w_u, U, _ = res
        n = prob.n
        rng = np.random.default_rng(0)
        k = min(args.check_slabs, n)
        slabs = sorted(set(list(range(min(16, k))) + list(rng.choice(n, size=max(0, k - 16),
                                                                            replace=False))))
        t0 = time.perf_counter()
        rep = osolve.rel_error(prob, w_u.cpu().numpy(), [u.cpu().numpy() for u in U], slabs=slabs)
        parity = {"rel_l2_sampled": rep["rel_l2"], "rel_residual_sampled": rep["rel_residual"],
                  "slabs": rep["slabs"], "gate": 10 * prob.eps,
                  "pass": bool(rep["rel_l2"] <= 10 * prob.eps)}
        log(f"[bench] oracle check on {rep['slabs']} slabs: {parity} "
            f"({time.perf_counter() - t0:.1f}s)")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(prob)
        log(f"[bench] cpu baseline {cpu}")

    fp64_value = value
    if batched is not None:
        value = batched["solves_per_s"]
        batched["vs_fp64_single"] = value / fp64_value
    rec = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.batch}x sine_n1024_rank10 batched (seeds 100..)"
                                if batched is not None else wname),
                   "n": prob.n, "rank_y": prob.rank, "alpha": prob.alpha,
                   "beta": prob.beta, "gamma": prob.gamma, "eps": prob.eps,
                   "path": "fp64, concurrent streams" if batched is not None else "fp64",
                   "setup_s": setup_s},
        "roofline": roof, "cpu_baseline": cpu, "parity": parity, "solve_info": info,
        "fp64_single": {"solves_per_s": fp64_value, "ms_per_solve": 1e3 * elapsed / args.steps},
        "batched": batched, "mixed_single": mixed,
    }
    print(json.dumps(rec), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
