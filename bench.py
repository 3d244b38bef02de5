#!/usr/bin/env python
"""Throughput of the rank-truncated PCG solve on one MI355X.

A solve is Algorithm 1 of the paper (with the entry and exit transforms and
the Tucker-to-canonical output) for the control equation
(beta A^-alpha + (gamma/beta) A^alpha) u = y and one design function, with the
plan (eigenpairs, separable operator and preconditioner) built beforehand and
the inputs resident in HBM.

The headline value: a step is one batched call (fc_solve_batched, concurrent
streams) solving 64 independent problems at n = 1024 per mode,
a_l(x) = 1 + 0.9 sin(4 pi x + phi_l) with seeded phases, rank-10 Gaussian-bump
designs, alpha = 0.5, beta = 1e-4, gamma = 1, eps = 1e-6, FP64; value =
solves/sec over the timed steps.  Also measured: the plain FP64 path one solve
at a time, the mixed-precision path (single and batched), and a batch of
uneven sizes (n from 64 to 2048).

Prints one JSON line with the roofline of the dominant single kernel of a
solve (the larger timed share of the Gram-Schmidt panel kernel and the
symmetric eigensolver; the GEMM family beside it), each launch timed with HIP
events on its stream in the single-solve timed region, the CPU oracle timed
on a bounded sample on this host, and the oracle error of sampled results.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The batched call runs 16 solves on 16 streams; HIP maps streams onto its
# hardware queues (4 by default), so ask for at least one queue per stream.
# Read by the HIP runtime when it initialises, i.e. before torch touches the GPU.
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
except ValueError:
    _hwq = 0
if _hwq < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

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


def host_info():
    """CPU model, logical CPUs and the BLAS the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = max(d.get("num_threads", 1) for d in info)
    except Exception:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas,
            "blas_threads": int(threads)}


def _median_iqr(xs):
    q = np.percentile(np.asarray(xs), [25, 50, 75])
    return float(q[1]), float(q[2] - q[0])


def cpu_full_timings(repeats=5):
    """The oracle's exact solve timed in full (setup: three LAPACK
    tridiagonal eigensolves; solve: entry transform, divide over the n^3
    grid, three mode products) at n = 32 and n = 256: median and IQR."""
    import workloads as wl
    from oracle import solve as osolve
    out = {}
    for name, prob in (("small_n32", wl.workload_small()),
                       ("quadratic_n256", wl.workload_quadratic(n=256, alpha=0.5))):
        ts, tt = [], []
        for _ in range(repeats):
            t0 = time.perf_counter()
            sp = osolve.Spectral(prob)
            t1 = time.perf_counter()
            osolve.solve_full(prob, sp)
            t2 = time.perf_counter()
            ts.append(t1 - t0)
            tt.append(t2 - t0)
        med, iqr = _median_iqr(tt)
        smed, siqr = _median_iqr(ts)
        out[name] = {"n": prob.n, "repeats": repeats, "s_per_solve_median": med, "s_iqr": iqr,
                     "setup_s_median": smed, "setup_s_iqr": siqr, "solves_per_s": 1.0 / med}
    return out


def cpu_baseline(prob, sample_slabs=8, repeats=3):
    """The oracle's exact solve at the headline size, timed on a bounded
    sample: full setup (three LAPACK tridiagonal eigensolves and the entry
    transform), then the divide and the mode-2/3 products for `sample_slabs`
    of the n mode-1 slabs and the mode-1 product for the same share of
    columns, extrapolated to all n slabs; median (and IQR) over `repeats`."""
    from oracle import solve as osolve
    hi = host_info()
    n = prob.n
    totals = []
    for _ in range(repeats):
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
        totals.append(t_setup + scale * (t_slabs + t_mode1))
    med, iqr = _median_iqr(totals)
    return {
        "value": 1.0 / med, "unit": "solves/s", "cores": hi["blas_threads"], "kind": "oracle",
        "sample": (f"oracle exact solve at n={n}: setup timed in full, divide + mode-2/3 products "
                   f"timed on {sample_slabs} of {n} mode-1 slabs and the mode-1 product on the "
                   f"same share of columns, extrapolated x{n / sample_slabs:.0f}; median "
                   f"{med:.1f}s per solve (IQR {iqr:.2f}s over {repeats} repeats)"),
        "s_per_solve_median": med, "s_iqr": iqr, "host": hi,
    }


def build_plans(api, probs, precision=0, threads=16):
    """Plans for `probs`, built concurrently on host threads."""
    import threading
    plans = [None] * len(probs)
    errors = []

    def build(i):
        p = probs[i]
        try:
            plans[i] = api.Plan(p.n, p.a, p.alpha, p.beta, p.gamma, p.eps, precision=precision)
        except Exception as e:  # reported after the join
            errors.append(e)

    idx = list(range(len(probs)))
    th = [threading.Thread(target=lambda t=t: [build(i) for i in idx[t::threads]])
          for t in range(threads)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    if errors:
        raise errors[0]
    return plans


def batch_io(api, torch, dev, probs, cap):
    inputs = [(torch.from_numpy(np.asarray(p.w)).to(dev),
               [api.to_device_colmajor(y, dev) for y in p.Y]) for p in probs]
    outs = [(torch.empty(cap, dtype=torch.float64, device=dev),
             [torch.empty((cap, p.n), dtype=torch.float64, device=dev).t() for _ in range(3)])
            for p in probs]
    return inputs, outs


KERNELS = {0: "gemm_kernel / gemm_multi_kernel (short-reduction LDS-tiled FP64 MFMA GEMMs)",
           1: "panel_mgs_kernel (Gram-Schmidt panel, one workgroup)",
           2: "tdeig_*_kernel (symmetric eigensolver: tridiagonalisation, multisection, inverse "
              "iteration, clusters, back-transformation; five launches per call)",
           3: "stream_kernel + stream_reduce_kernel (mode transforms V^T Y, V Z on FP64 MFMA)",
           4: "gram_kernel / gram_multi_kernel / sgram_multi_kernel (long-reduction FP64 MFMA: "
              "Gram-type products, scaled Grams Z^T diag(d) X, core contractions)",
           5: "kron_apply_kernel (fused sum_q diag(D[:,q]) Z T^q on FP64 MFMA)"}
# names of the traffic records (profiles/*.md) of each kind: HBM bytes per
# launch of the family (an eigensolver call is five dispatches, a transform
# group two)
KERNEL_NAMES = {0: "short_gemm", 1: "panel_mgs_kernel", 2: "eigensolver", 3: "mode_transform",
                4: "long_gram", 5: "kron_apply_kernel"}
KIND_KEYS = {0: "short_gemm", 1: "gram_schmidt_panel", 2: "eigensolver", 3: "mode_transform",
             4: "long_gram", 5: "kron_apply"}


def kernel_profile(lib, check, kind):
    """(launches, total ms, algorithmic flops, algorithmic bytes) of one
    profile kind; kind -1: the whole product family (fc_profile_gemm_read)."""
    launches, ms, flops, byts = C.c_long(), C.c_double(), C.c_double(), C.c_double()
    if kind < 0:
        check(lib().fc_profile_gemm_read(C.byref(launches), C.byref(ms), C.byref(flops),
                                         C.byref(byts)), "fc_profile_gemm_read")
    else:
        check(lib().fc_profile_kernel_read(kind, C.byref(launches), C.byref(ms), C.byref(flops),
                                           C.byref(byts)), "fc_profile_kernel_read")
    return launches.value, ms.value, flops.value, byts.value


def roofline(kind, launches, ms, flops, byts):
    """Roofline of one kernel family from HIP-event timings: the algorithmic
    work per launch over the mean launch duration, against the HBM roof when
    the arithmetic intensity is below the FP64 ridge point (always for the
    mode transforms, whose V_l read dominates), else the FP64 matrix-core
    roof."""
    per_launch_s = (ms / 1e3) / max(launches, 1)
    fl_launch = flops / max(launches, 1)
    by_launch = byts / max(launches, 1)
    ai = flops / max(byts, 1.0)
    if ai >= PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9) and kind != 3:
        # above the ridge: the FP64 matrix cores for the GEMMs; the eigensolver
        # computes on the FP64 vector units (same 78.6 TFLOP/s peak)
        achieved = fl_launch / per_launch_s / 1e12
        roof = {"bound": "alu" if kind == 2 else "mfma", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None}
    else:
        achieved = by_launch / per_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof.update({"kernel": KERNELS[kind], "launches_timed": launches,
                 "avg_launch_us": per_launch_s * 1e6, "flops_per_launch": fl_launch,
                 "bytes_per_launch": by_launch, "arith_intensity": ai})
    return roof


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if the kernel source is unchanged since
    it was taken (the record carries the SHA-256 of the kernel source); else
    None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2006_09314_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if line.startswith("traffic-record: "):
                    rec = json.loads(line[len("traffic-record: "):])
                    if rec.get("kernel") != kernel:
                        continue
                    if rec.get("kernel_source_sha256") == digest:
                        return rec["hbm_bytes_per_launch"], os.path.basename(path)
                    return None, f"{os.path.basename(path)} (stale: kernel source changed)"
    return None, "no counter record"


def sampled_parity(prob, w_u, U, k, seed):
    from oracle import solve as osolve
    n = prob.n
    rng = np.random.default_rng(seed)
    slabs = sorted(set(list(range(min(k // 2, n))) +
                       list(rng.choice(n, size=min(n, k - k // 2), replace=False))))
    rep = osolve.rel_error(prob, w_u.cpu().numpy(), [u.cpu().numpy() for u in U], slabs=slabs)
    return {"rel_l2_sampled": rep["rel_l2"], "rel_residual_sampled": rep["rel_residual"],
            "slabs": rep["slabs"], "gate": 10 * prob.eps,
            "pass": bool(rep["rel_l2"] <= 10 * prob.eps)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6,
                    help="timed batched steps (one step = one batched call over --batch problems)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", default="sine1024", help="single-solve workload")
    ap.add_argument("--single-steps", type=int, default=5)
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--no-mixed-batch", action="store_true")
    ap.add_argument("--uneven", type=int, default=16,
                    help="problems in the uneven-size batched measurement (0 disables it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--check-slabs", type=int, default=24)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a "
                         "known-size reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: each solve "
              "runs on a single device, and independent problems would be spread over GPUs "
              "one process per GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    from paper_2006_09314_amd import api
    from paper_2006_09314_amd._lib import check, lib

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.copy_mib > 0:
        nel = args.copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] reference copy of {args.copy_mib} MiB done")
        del src, dst

    # ---- FP64, one solve at a time (the plain path) -------------------------
    prob, wname = make_workload(args.workload)
    log(f"[bench] single workload {wname}: n={prob.n} rank_y={prob.rank} alpha={prob.alpha} "
        f"beta={prob.beta} eps={prob.eps}")
    t0 = time.perf_counter()
    plan = api.Plan(prob.n, prob.a, prob.alpha, prob.beta, prob.gamma, prob.eps)
    setup_s = time.perf_counter() - t0
    w = torch.from_numpy(np.asarray(prob.w)).to(dev)
    Y = [api.to_device_colmajor(y, dev) for y in prob.Y]
    cap = 8192
    out = (torch.empty(cap, dtype=torch.float64, device=dev),
           [torch.empty((cap, prob.n), dtype=torch.float64, device=dev).t() for _ in range(3)])
    res = plan.solve(w, Y, cap_u=cap, out=out)
    tuning = plan.tuning()
    log(f"[bench] setup {setup_s:.2f}s; autotuner {tuning}; warm-up solve {res[2]}")
    torch.cuda.synchronize()
    check(lib().fc_profile_gemm(1), "fc_profile_gemm")
    t0 = time.perf_counter()
    for _ in range(args.single_steps):
        res = plan.solve(w, Y, cap_u=cap, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    check(lib().fc_profile_gemm(0), "fc_profile_gemm")
    kinds = sorted(KERNELS)
    profs = {k: kernel_profile(lib, check, k) for k in kinds}
    # the dominant kernel of the solve: the kernel family with the largest
    # share of the timed solves (HIP events around every launch)
    dom = max(kinds, key=lambda k: profs[k][1])
    roof = roofline(dom, *profs[dom])
    roof["measured_in"] = ("FP64 single-solve timed region, one stream (under concurrent streams "
                           "HIP events time queueing, not kernel duration)")
    roof["share_of_solve"] = (profs[dom][1] / 1e3) / el
    roof["traffic"], roof["traffic_source"] = recorded_traffic(KERNEL_NAMES[dom])
    others = {}
    for k in kinds:
        if k == dom:
            continue
        r = roofline(k, *profs[k])
        r["share_of_solve"] = (profs[k][1] / 1e3) / el
        r["per_solve_bytes"] = profs[k][3] / args.single_steps
        r["per_solve_flops"] = profs[k][2] / args.single_steps
        r["traffic"], r["traffic_source"] = recorded_traffic(KERNEL_NAMES[k])
        others[KIND_KEYS[k]] = r
    roof["other_kernels"] = others
    # algorithmic work of one solve over all timed kernel families (for the
    # roofline of the batched step)
    solve_flops = sum(profs[k][2] for k in kinds) / args.single_steps
    solve_bytes = sum(profs[k][3] for k in kinds) / args.single_steps
    profs[0] = kernel_profile(lib, check, -1)   # the whole product family (kinds 0, 3, 4, 5)
    sl = profs[0][0]
    sms = profs[0][1]
    single = {"solves_per_s": args.single_steps / el, "ms_per_solve": 1e3 * el / args.single_steps,
              "info": res[2], "gemm_launches_per_solve": sl / args.single_steps,
              "gemm_share_of_solve": (sms / 1e3) / el}
    log(f"[bench] FP64 single: {single['solves_per_s']:.2f} solves/s")
    if not args.no_check:
        single["parity"] = sampled_parity(prob, res[0], res[1], args.check_slabs, 0)
        log(f"[bench] FP64 single parity {single['parity']}")

    # ---- mixed precision, one solve at a time --------------------------------
    mixed = None
    if args.mixed_steps > 0:
        mplan = api.Plan(prob.n, prob.a, prob.alpha, prob.beta, prob.gamma, prob.eps, precision=1)
        res_m = mplan.solve(w, Y, cap_u=cap, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.mixed_steps):
            res_m = mplan.solve(w, Y, cap_u=cap, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mixed = {"solves_per_s": args.mixed_steps / el,
                 "ms_per_solve": 1e3 * el / args.mixed_steps, "info": res_m[2]}
        if not args.no_check:
            mixed["parity"] = sampled_parity(prob, res_m[0], res_m[1], 20, 2)
        log(f"[bench] mixed single: {mixed}")
        mplan.close()
    plan.close()

    # ---- batched FP64 at n = 1024: the timed region of the headline value ----
    probs = wl.workload_batched_uniform(count=args.batch, n=1024)
    log(f"[bench] batched: {len(probs)} problems at n=1024 (sine family, seeds 100..); "
        "building plans ...")
    t0 = time.perf_counter()
    plans = build_plans(api, probs)
    bsetup = time.perf_counter() - t0
    inputs, outs = batch_io(api, torch, dev, probs, 1024)
    for _ in range(args.warmup):
        res_b = api.solve_batched(plans, inputs, cap_u=1024, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        res_b = api.solve_batched(plans, inputs, cap_u=1024, outs=outs)   # returns when all are done
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps * len(probs) / elapsed
    # the batched step as a whole: the algorithmic work of the timed kernel
    # families per solve (single-solve profile) times the solves per second
    # of the step, against the FP64 peak and the HBM roof
    step_tflops = solve_flops * value / 1e12
    step_gbs = solve_bytes * value / 1e9
    roof["step"] = {"what": "timed batched step, all kernel families, algorithmic work per solve x "
                            "solves/s",
                    "flops_per_solve": solve_flops, "bytes_per_solve": solve_bytes,
                    "achieved_tflops": step_tflops, "frac_fp64_peak": step_tflops / PEAK_FP64_TFLOPS,
                    "achieved_gbs": step_gbs, "frac_hbm": step_gbs / PEAK_HBM_GBS}
    iters = [r[2]["iterations"] for r in res_b]
    batched = {"problems": len(probs), "setup_s": bsetup, "solves_per_s": value,
               "streams": int(os.environ.get("FC_BATCH_STREAMS", "16")),
               "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
               "iterations_min_max": [min(iters), max(iters)],
               "step_s": [round(x, 4) for x in step_s],
               "vs_fp64_single": value / single["solves_per_s"]}
    log(f"[bench] batched FP64: {args.steps} x {len(probs)} solves in {elapsed:.2f}s -> "
        f"{value:.2f} solves/s")
    if not args.no_check:
        batched["parity"] = [dict(problem=i, **sampled_parity(probs[i], res_b[i][0], res_b[i][1],
                                                              16, 10 + i))
                             for i in (0, len(probs) - 1)]
        log(f"[bench] batched parity {batched['parity']}")
    for p_ in plans:
        p_.close()

    # ---- batched mixed precision on the same problems ------------------------
    mixed_batched = None
    if not args.no_mixed_batch:
        plans = build_plans(api, probs, precision=1)
        res_mb = api.solve_batched(plans, inputs, cap_u=1024, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res_mb = api.solve_batched(plans, inputs, cap_u=1024, outs=outs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mixed_batched = {"problems": len(probs), "solves_per_s": args.steps * len(probs) / el,
                         "refinements_min_max": [min(r[2]["refinements"] for r in res_mb),
                                                 max(r[2]["refinements"] for r in res_mb)]}
        if not args.no_check:
            mixed_batched["parity"] = sampled_parity(probs[0], res_mb[0][0], res_mb[0][1], 16, 20)
        log(f"[bench] batched mixed: {mixed_batched}")
        for p_ in plans:
            p_.close()
    del inputs, outs

    # ---- batched FP64, uneven sizes and ranks (n in 64..2048) ----------------
    uneven = None
    if args.uneven > 0:
        uprobs = wl.workload_batched(count=args.uneven)
        torch.cuda.synchronize()
        t_setup = time.perf_counter()
        plans = build_plans(api, uprobs)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        uin, uout = batch_io(api, torch, dev, uprobs, 2048)
        res_u = api.solve_batched(plans, uin, cap_u=2048, outs=uout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_u = api.solve_batched(plans, uin, cap_u=2048, outs=uout)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ns = [p.n for p in uprobs]
        uneven = {"problems": len(uprobs), "n_values": sorted(set(ns)),
                  "solves_per_s": len(uprobs) / el, "s_per_batch": el,
                  "setup_s": t_setup,
                  "solves_per_s_with_setup": len(uprobs) / (el + t_setup)}
        if not args.no_check:
            big = int(np.argmax(ns))
            uneven["parity_largest"] = dict(problem=big, n=ns[big], **sampled_parity(
                uprobs[big], res_u[big][0], res_u[big][1], 8, 30))
        log(f"[bench] batched uneven: {uneven}")
        for p_ in plans:
            p_.close()
        del uin, uout

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(prob)
        cpu["full_solves"] = cpu_full_timings()
        log(f"[bench] cpu baseline {cpu}")

    rec = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(probs)}x sine_n1024_rank10 batched (seeds 100..)",
                   "step": f"one batched call solving {len(probs)} problems",
                   "n": 1024, "rank_y": 10, "alpha": 0.5, "beta": 1e-4, "gamma": 1.0,
                   "eps": 1e-6, "path": "fp64, concurrent streams"},
        "roofline": roof, "cpu_baseline": cpu, "autotune": tuning,
        "fp64_single": single, "batched": batched, "mixed_single": mixed,
        "mixed_batched": mixed_batched, "batched_uneven": uneven,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
