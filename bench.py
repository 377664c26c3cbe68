#!/usr/bin/env python3
"""Benchmark: cooperative CG solves per second on one MI355X.

Default workload (--mode single; one "step" = one complete solve): dense SPD
A = Q diag(lam) Q^T with n = 8192, lam log-uniform in [1, 1e4] (condition number
1e4 exactly), b and the p = 8 starting points N(0,1), seeded; stop when the best
agent's explicit FP64 relative residual is <= 1e-10.  Inputs are resident in HBM
before timing starts.  --kind gram selects A = M^T M / n + sigma I instead, and
--prec fp32 / bf16x2 the mixed-precision refinement modes.

Printed: ONE JSON line with solves/s, ms per solve, p50/p99 solve latency, the
A.D kernel's achieved HBM bandwidth against the 8 TB/s peak (HIP events around
every A.D launch, on the library's stream, inside the timed region), and the
oracle's throughput on the host cores on a bounded sample of the same workload.

Other modes (their own JSON line each):
  --mode batched  many independent systems in one ccg_solve_batched call (n
                  log-uniform in [64, 4096], p in {2, 4, 8}, kappa log-uniform in
                  [1e2, 1e5], FP32 A + FP64 refinement); one step = the whole batch.
  --mode served   Poisson arrivals into the continuous-batching service (n
                  log-uniform in [128, 16384], p = 4, kappa log-uniform in
                  [1e2, 1e6], precision drawn from fp64 / fp32 / bf16x2, A in pinned
                  host memory, upload inside the latency); reports p50/p99 latency.
  --mode paper    the paper's own experiment (Sec. 5): A = U diag(lam) U^T with U
                  Haar, lam uniform in [1, 1e6], b and the starting points uniform in
                  [-10, 10], n from 1000 to 25000, cCG with p = 3 against CG (p = 1)
                  from the first of the three starting points, stop when the best
                  agent's residual norm is <= 1e-3, read both as absolute and as
                  relative to ||b||; reports the mean block steps per n, their ratio
                  CG / cCG and the log-log slope of cCG's steps against n, beside the
                  paper's Table 4 ratios and Fig. 5 slope.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/s + A·D HBM GB/s vs peak at rel. residual 1e-10; p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed solves")
    ap.add_argument("--warmup", type=int, default=2, help="untimed solves")
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--kappa", type=float, default=1e4)
    ap.add_argument("--seed", type=int, default=None,
                    help="base seed of the single-system inputs (default: the fixed base seed)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x2"])
    ap.add_argument("--cpu-sample-steps", type=int, default=12,
                    help="block steps of the oracle timed on the host (0: skip)")
    ap.add_argument("--profile-all", action="store_true",
                    help="time every A.D launch (all block steps launched directly)")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not time A.D launches (graphs carry no event nodes)")
    ap.add_argument("--mode", default="single", choices=["single", "batched", "served", "paper", "psweep", "tier"])
    ap.add_argument("--psweep", default="1,2,3,4,5,6,8,10,12,16,20,24,32",
                    help="psweep mode: agent counts")
    ap.add_argument("--paper-sizes", default="1000,1500,2000,2500,3000,3500,4000,4500,5000,6000,7000,8000,"
                                             "9000,10000,11000,12000,13000,14000,15000,16000,17000,18000,"
                                             "19000,20000,21000,22000,23000,24000,25000",
                    help="paper mode: system sizes")
    ap.add_argument("--paper-ics", type=int, default=0,
                    help="paper mode: starting blocks per size (0: 20 below n = 5000, 10 from there, "
                         "as in Sec. 5)")
    ap.add_argument("--paper-tol-sweep", action="store_true",
                    help="paper mode: only the tolerance sweep of Table 2 (n = 8000, tol 1e-3 .. 1e-9)")
    ap.add_argument("--kind", default="spectrum", choices=["spectrum", "gram"],
                    help="single mode: Q diag(lam) Q^T, or M^T M / n + sigma I")
    ap.add_argument("--count", type=int, default=1024, help="batched mode: systems per batch")
    ap.add_argument("--requests", type=int, default=1000, help="served mode: timed requests")
    ap.add_argument("--pool", type=int, default=64, help="served mode: distinct matrices")
    ap.add_argument("--n-hi", type=int, default=16384, help="served mode: largest n")
    ap.add_argument("--rate-frac", type=float, default=0.5,
                    help="served mode: arrival rate as a fraction of the closed-loop rate")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="served mode: arrivals per second (0: --rate-frac x the measured closed-loop rate)")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="served mode: HBM budget")
    ap.add_argument("--no-compare-fp64", dest="compare_fp64", action="store_false",
                    help="served mode: skip the plain FP64 comparison")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="time read-only streams of the A.D traffic shape at --n (ccg_stream_probe)")
    ap.add_argument("--dump", default=None, help="served mode: write per-request records (JSON) here")
    ap.add_argument("--single-fp64", action="store_true",
                    help="batched mode: time the plain FP64 baseline instead (every 8th system, one "
                         "ccg_solve at a time)")
    ap.add_argument("--no-c3", dest="c3", action="store_false",
                    help="single mode: skip the n = 32768 sub-record (FP64 and BF16x2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (3 times) and exit: the "
                         "known-size kernel that scales hardware byte counters")
    return ap.parse_args()


def kernel_source_sha(prec: str) -> str:
    """sha256 over the sources that decide the A.D kernel of a precision: the device
    templates, the precision's translation unit and the tile-width table."""
    import hashlib
    csrc = os.path.join(HERE, "paper_1204_0069_amd", "csrc")
    tag = {"fp64": "f64", "fp32": "f32", "bf16x2": "bf16"}[prec]
    h = hashlib.sha256()
    for name in ("ccg_kernels.h", f"ccg_ad_{tag}.hip", "ccg_tune_table.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(n: int, p: int, prec: str):
    """HBM bytes per A.D launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    (profiles/), or None when no run covers this workload or the kernel source has
    changed since the counters were taken."""
    path = os.path.join(HERE, "profiles", f"k_ad_{prec}_n{n}_p{p}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "*", "`", " ")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    sha = kernel_source_sha(prec)
    if rec.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in rec:
        return None
    return int(rec["traffic_bytes_per_launch"])


def copy_calibration(mib: int):
    """A plain device copy of known size, for reading FETCH_SIZE / WRITE_SIZE."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the solver has no "
                                   "multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.stream_ceiling:
        return stream_ceiling(args)

    if args.mode == "batched":
        return run_batched(args)
    if args.mode == "served":
        return run_served(args)
    if args.mode == "paper":
        return run_paper(args)
    if args.mode == "psweep":
        return run_psweep(args)
    if args.mode == "tier":
        return run_tier(args)

    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_PROFILE, CCG_PROFILE_SAMPLED, Context

    dev = "cuda:0"
    n, p = args.n, args.p
    seed = ci.BASE_SEED if args.seed is None else args.seed
    if args.kind == "gram":
        A = ci.spd_gram(n, args.kappa, ci.item_seed("G", seed, base=n), device=dev)
    else:
        A = ci.spd_spectrum(n, args.kappa, ci.item_seed("A", seed, base=n), device=dev)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", seed, base=n)), device=dev)
    X0 = torch.as_tensor(ci.normal_block(n, p, ci.item_seed("X0", seed, base=n)), device=dev)
    torch.cuda.synchronize()

    ctx = Context(0)
    flags = 0 if args.no_profile else (CCG_PROFILE if args.profile_all else CCG_PROFILE_SAMPLED)
    t = time_solves(ctx, A, b, X0, args.tol, args.prec, args.steps, args.warmup, flags,
                    graph_rate=not args.no_profile)
    iters = [i["iters"] for i in t["infos"]]
    roofline = None
    if t["ad_launches"] > 0:
        roofline = roofline_record(n, p, args.prec, t["ad_ms"], t["ad_launches"], args.profile_all)
    error = result_errors(ctx, A, b, X0, t["X"], t["infos"][-1], args.tol, args.prec)

    cpu = None
    if args.cpu_sample_steps > 0:
        cpu = cpu_baseline(A, b, X0, args.cpu_sample_steps, float(np.mean(iters)))

    lat_ms = np.array(t["lat"]) * 1e3
    out = {
        "metric": METRIC,
        "value": round(args.steps / t["total"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t["total"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x2": "bf16x2"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"dense SPD n={n}, kappa={args.kappa:g} "
                               f"({'log-uniform spectrum' if args.kind == 'spectrum' else 'M^T M/n + sigma I'}), "
                               f"p={p} agents, {args.prec.upper()} A, tol {args.tol:g}",
                   "n": n, "p": p, "kappa": args.kappa, "tol": args.tol, "prec": args.prec, "seed": seed,
                   "kind": args.kind},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "solves_per_s_graph": None if t["graph_rate"] is None else round(t["graph_rate"], 4),
        "iters_per_solve": float(np.mean(iters)),
        "restarts": int(sum(i["restarts"] for i in t["infos"])),
        "rel_res": t["rel_res"],
        "status": t["infos"][-1]["status_name"],
        "error": error,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    del A, b, X0, t
    torch.cuda.empty_cache()
    if args.c3 and args.n == 8192 and args.kind == "spectrum" and args.prec == "fp64":
        out["c3"] = run_c3(ctx, args)
    print(json.dumps(out))
    ctx.close()


def time_solves(ctx, A, b, X0, tol, prec, steps, warmup, flags, graph_rate=True):
    """Warm-up solves, then `steps` timed solves (A.D launches timed per `flags`), then
    optionally the same solves from captured graphs with no events.  Inputs resident
    in HBM; the timed region is bracketed by device synchronisations."""
    import torch
    for _ in range(warmup):
        ctx.solve(A, b, X0, tol, 100000, prec=prec, flags=flags)
    ctx.kernel_time(reset=True)
    lat, infos = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        X, info = ctx.solve(A, b, X0, tol, 100000, prec=prec, flags=flags)
        lat.append(time.perf_counter() - s0)
        infos.append(info)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ad_ms, ad_launches = ctx.kernel_time(reset=True)
    g_rate = None
    if graph_rate and flags:
        ctx.solve(A, b, X0, tol, 100000, prec=prec)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(steps):
            ctx.solve(A, b, X0, tol, 100000, prec=prec)
        torch.cuda.synchronize()
        g_rate = steps / (time.perf_counter() - g0)
    # explicit residual of the last result, independent of the library (rocBLAS)
    T = b[:, None] - A @ X
    rel = (torch.linalg.norm(T, dim=0) / torch.linalg.norm(b)).cpu().numpy()
    return {"lat": lat, "infos": infos, "total": total, "ad_ms": ad_ms, "ad_launches": ad_launches,
            "graph_rate": g_rate, "X": X, "rel_res": float(rel.min())}


def roofline_record(n, p, prec, ad_ms, ad_launches, every):
    s_a = {"fp64": 8, "fp32": 4, "bf16x2": 4}[prec]
    s_v = 8 if prec == "fp64" else 4
    bytes_per_launch = n * n * s_a + 2 * n * p * s_v
    avg_s = ad_ms / 1e3 / ad_launches
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(n, p, prec), "traffic_unit": "B/launch",
            "kernel": "k_ad",
            "avg_launch_us": round(avg_s * 1e6, 2), "launches": ad_launches,
            "timed": ("every A.D launch" if every else
                      "the A.D launches of every 4th round of block steps"),
            "bytes_per_launch": bytes_per_launch}


def result_errors(ctx, A, b, X0, X, info, tol, prec):
    """Per-result error of the reported (best) agent: against x* = A^{-1} b (FP64 LU,
    rocSOLVER through torch), and for the low-precision modes against the result of
    the same solve in FP64 mode (one more, untimed, solve)."""
    import torch
    xs = torch.linalg.solve(A, b)
    j = info["best_agent"]
    nx = torch.linalg.norm(xs)
    err = {"vs_xstar": float(torch.linalg.norm(X[:, j] - xs) / nx),
           "vs_xstar_max_agent": float((torch.linalg.norm(X - xs[:, None], dim=0) / nx).max()),
           "xstar": "torch.linalg.solve (FP64 LU)"}
    if prec != "fp64":
        X64, i64 = ctx.solve(A, b, X0, tol, 100000)
        err["vs_fp64_mode"] = float(torch.linalg.norm(X[:, j] - X64[:, i64["best_agent"]]) /
                                    torch.linalg.norm(X64[:, i64["best_agent"]]))
    del xs
    return err


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(A, b, X0, sample_steps, steps_per_gpu_solve):
    """The oracle on the host on `sample_steps` block steps of the same system: one
    thread (the oracle as built for the tests), and the OpenMP build of the same
    source (the same bits) on the threads OMP_NUM_THREADS allows."""
    import numpy as np

    import oracle
    An = A.cpu().numpy()
    bn = b.cpu().numpy()
    Xn = X0.cpu().numpy()
    n, p = Xn.shape
    steps_per_solve = steps_per_gpu_solve + 2.0          # + initial and confirming residuals
    rec = {}
    for name, lib in (("one", None), ("all", oracle.all_cores())):
        c0 = time.perf_counter()
        oracle.ccg(An, bn, Xn, tol=0.0, maxit=sample_steps, lib=lib)
        c1 = time.perf_counter()
        per_step = (c1 - c0) / (sample_steps + 1)          # + the initial residual pass
        rec[name] = (per_step, c1 - c0)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    per1, t1 = rec["one"]
    perA, tA = rec["all"]
    return {"value": round(1.0 / (per1 * steps_per_solve), 6), "unit": "solves/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{sample_steps} block steps of the same n={n}, p={p} system "
                      f"({t1:.1f} s, {per1:.3f} s per A stream); solves/s = 1 / "
                      f"(s per step x {steps_per_solve:.0f} steps per solve)",
            "all_cores": {"value": round(1.0 / (perA * steps_per_solve), 6), "unit": "solves/s",
                          "cores": threads,
                          "sample": f"the same {sample_steps} steps, OpenMP build over rows "
                                    f"({tA:.1f} s, {perA:.3f} s per A stream)"},
            "cpu_model": cpu_model(), "host_cores": os.cpu_count()}


def run_c3(ctx, args):
    """n = 32768, p = 8, A = M^T M / n + sigma I (cond 1e3), tol 1e-10: FP64 and
    BF16 hi+lo with FP64 refinement (the largest single-GPU workload; A is 8 GiB, far
    beyond the 256 MB MALL)."""
    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_PROFILE_SAMPLED
    dev = "cuda:0"
    n, p, kappa = 32768, 8, 1e3
    A = ci.spd_gram(n, kappa, ci.item_seed("G", ci.BASE_SEED, base=n), device=dev)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", ci.BASE_SEED, base=n)), device=dev)
    X0 = torch.as_tensor(ci.normal_block(n, p, ci.item_seed("X0", ci.BASE_SEED, base=n)), device=dev)
    torch.cuda.synchronize()
    rec = {"workload": f"dense SPD n={n}, M^T M/n + sigma I (cond {kappa:g}), p={p}, tol {args.tol:g}"}
    xs = torch.linalg.solve(A, b)
    X64 = None
    for prec in ("fp64", "bf16x2"):
        t = time_solves(ctx, A, b, X0, args.tol, prec, 2, 1, CCG_PROFILE_SAMPLED, graph_rate=False)
        info = t["infos"][-1]
        j = info["best_agent"]
        r = {"solves_per_s": round(2 / t["total"], 4), "iters_per_solve": float(np.mean([i["iters"] for i in t["infos"]])),
             "rel_res": t["rel_res"], "status": info["status_name"],
             "error_vs_xstar": float(torch.linalg.norm(t["X"][:, j] - xs) / torch.linalg.norm(xs))}
        if t["ad_launches"] > 0:
            rr = roofline_record(n, p, prec, t["ad_ms"], t["ad_launches"], False)
            r["ad_frac"] = rr["frac"]
            r["ad_avg_launch_us"] = rr["avg_launch_us"]
        if prec == "fp64":
            X64 = t["X"][:, j].clone()
        else:
            r["error_vs_fp64_mode"] = float(torch.linalg.norm(t["X"][:, j] - X64) / torch.linalg.norm(X64))
        rec[prec] = r
        print(json.dumps({"progress": "c3", "prec": prec}), file=sys.stderr, flush=True)
    del A, b, X0, xs
    torch.cuda.empty_cache()
    return rec


# The paper's numbers for its own experiment (Sec. 5; Core2Quad, p = 3, tol 1e-3):
# Table 4's iteration ratios CG / cCG per n, the mean of that column, and the slope
# of the least-squares line through log(cCG iterations) against log(n) of Fig. 5.
PAPER_TABLE4_RATIO = {1000: 1.79, 1500: 1.40, 2000: 1.66, 2500: 1.46, 3000: 1.57, 3500: 1.67, 4000: 1.55,
                      4500: 1.65, 5000: 1.78, 6000: 1.34, 7000: 1.33, 8000: 1.24, 9000: 1.80, 10000: 1.96,
                      11000: 1.61, 12000: 1.74, 13000: 1.51, 14000: 1.79, 15000: 1.85, 16000: 1.58,
                      17000: 1.53, 18000: 1.65, 19000: 1.71, 20000: 1.76, 21000: 1.67, 22000: 1.62,
                      23000: 1.38, 24000: 1.69, 25000: 1.81}
PAPER_MEAN_RATIO = 1.62
PAPER_ITER_SLOPE = 0.501
# Table 2: n = 8000, 10 starting points: (tol, CG iterations, cCG iterations)
PAPER_TABLE2 = [(1e-3, 372.2, 299.7), (1e-4, 414.0, 319.4), (1e-5, 444.9, 335.0), (1e-6, 476.8, 352.7),
                (1e-7, 510.7, 336.2), (1e-8, 538.4, 373.5), (1e-9, 559.7, 381.2)]


def _paper_system(n, dev):
    """A, b of the paper's experiment at size n (Sec. 5): U Haar, lam uniform in
    [1, 1e6], b uniform in [-10, 10]; seeded by n."""
    import torch

    import ccg_inputs as ci
    A = ci.spd_spectrum(n, 1e6, ci.item_seed("P", ci.BASE_SEED, base=n), lam_dist="uniform", device=dev)
    b = torch.as_tensor(ci.uniform_block(n, 0, ci.item_seed("pb", ci.BASE_SEED, base=n)), device=dev)
    return A, b


def _paper_start(n, ic, dev):
    import torch

    import ccg_inputs as ci
    return torch.as_tensor(ci.uniform_block(n, 3, ci.item_seed("pX0", ic, base=n)), device=dev)


def run_paper(args):
    """The paper's experiment on the GPU: block steps of cCG (p = 3) and CG (p = 1) to
    tol 1e-3, both readings of the tolerance.  One JSON line."""
    import numpy as np
    import torch

    from paper_1204_0069_amd import Context

    dev = "cuda:0"
    ctx = Context(0)
    if args.paper_tol_sweep:
        n = 8000
        A, b = _paper_system(n, dev)
        nb = float(torch.linalg.norm(b))
        rows = []
        for tol, cg_paper, ccg_paper in PAPER_TABLE2:
            row = {"tol": tol, "paper_cg_iters": cg_paper, "paper_ccg_iters": ccg_paper}
            for reading, t in (("abs", tol / nb), ("rel", tol)):
                it3, it1 = [], []
                for ic in range(10):
                    X0 = _paper_start(n, ic, dev)
                    it3.append(ctx.solve(A, b, X0, t, 10 ** 6)[1]["iters"])
                    it1.append(ctx.solve(A, b, X0[:, :1], t, 10 ** 6)[1]["iters"])
                row[reading] = {"cg_iters": float(np.mean(it1)), "ccg_iters": float(np.mean(it3)),
                                "ratio": float(np.mean(it1) / np.mean(it3))}
            rows.append(row)
            print(json.dumps({"progress": "tol", "tol": tol}), file=sys.stderr, flush=True)
        ctx.close()
        print(json.dumps({"mode": "paper_tol_sweep", "n": n, "kappa": 1e6, "starts": 10, "rows": rows,
                          "paper": "Table 2 (Sec. 5): mean iterations of CG and cCG (p = 3) at n = 8000"}))
        return
    sizes = [int(v) for v in args.paper_sizes.split(",") if v]
    rows = []
    t_all = time.perf_counter()
    for n in sizes:
        A, b = _paper_system(n, dev)
        nb = float(torch.linalg.norm(b))
        ics = args.paper_ics or (20 if n < 5000 else 10)
        row = {"n": n, "starts": ics, "paper_ratio": PAPER_TABLE4_RATIO.get(n)}
        for reading, t in (("abs", 1e-3 / nb), ("rel", 1e-3)):
            it3, it1, s3, s1 = [], [], [], []
            for ic in range(ics):
                X0 = _paper_start(n, ic, dev)
                c0 = time.perf_counter()
                _, i3 = ctx.solve(A, b, X0, t, 10 ** 6)
                c1 = time.perf_counter()
                _, i1 = ctx.solve(A, b, X0[:, :1], t, 10 ** 6)
                c2 = time.perf_counter()
                assert i3["status"] == 0 and i1["status"] == 0, (i3, i1)
                it3.append(i3["iters"])
                it1.append(i1["iters"])
                s3.append(c1 - c0)
                s1.append(c2 - c1)
            row[reading] = {"ccg_iters": float(np.mean(it3)), "cg_iters": float(np.mean(it1)),
                            "ratio": float(np.mean(it1) / np.mean(it3)),
                            "ccg_ms": round(1e3 * float(np.mean(s3)), 2),
                            "cg_ms": round(1e3 * float(np.mean(s1)), 2)}
        rows.append(row)
        print(json.dumps({"progress": n, "abs_ratio": round(row["abs"]["ratio"], 3),
                          "rel_ratio": round(row["rel"]["ratio"], 3)}), file=sys.stderr, flush=True)
        del A, b
        torch.cuda.empty_cache()
    ctx.close()
    ln = np.log([r["n"] for r in rows])
    summary = {}
    for reading in ("abs", "rel"):
        it = np.log([r[reading]["ccg_iters"] for r in rows])
        slope = float(np.polyfit(ln, it, 1)[0]) if len(rows) > 1 else None
        ratios = [r[reading]["ratio"] for r in rows]
        summary[reading] = {"mean_ratio": round(float(np.mean(ratios)), 3),
                            "iters_slope": None if slope is None else round(slope, 3)}
    print(json.dumps({"mode": "paper", "workload": "A = U diag(lam) U^T, U Haar, lam uniform in [1, 1e6], "
                                                   "b and X0 uniform in [-10, 10], p = 3 against p = 1, tol 1e-3",
                      "rows": rows, "summary": summary,
                      "paper": {"mean_ratio": PAPER_MEAN_RATIO, "iters_slope": PAPER_ITER_SLOPE,
                                "source": "Table 4 (iteration ratio per n) and Fig. 5 (slope), Sec. 5"},
                      "seconds": round(time.perf_counter() - t_all, 1)}))


def run_tier(args):
    """Single solves of small systems on the small-system tier (the default where it
    applies) and on the multi-workgroup path (CCG_NO_TIER): milliseconds per solve over
    10 solves after one warm-up, and per block step.  One JSON line."""
    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_NO_TIER, Context

    dev = "cuda:0"
    ctx = Context(0)
    rows = []
    for n, p, kappa in [(64, 4, 1e3), (96, 4, 1e3), (128, 4, 1e3), (256, 3, 1e3), (256, 8, 1e4), (512, 8, 1e4)]:
        A, b, X0 = (torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
                    for x in ci.system(n, p, kappa, seed=7))
        for prec in ("fp64", "fp32"):
            for fl in (0, CCG_NO_TIER):
                ctx.solve(A, b, X0, 1e-10, 100000, prec=prec, flags=fl)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(10):
                    X, info = ctx.solve(A, b, X0, 1e-10, 100000, prec=prec, flags=fl)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / 10
                rows.append({"n": n, "p": p, "prec": prec, "path": "multi" if fl else "default",
                             "ms": round(dt * 1e3, 3), "iters": info["iters"],
                             "us_per_step": round(dt * 1e6 / max(1, info["iters"]), 2)})
                print(json.dumps({"progress": "tier", **rows[-1]}), file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps({"mode": "tier", "rows": rows,
                      "note": "default = the small-system tier where n <= 96 and p <= 4, else the "
                              "multi-workgroup step; multi = CCG_NO_TIER"}))


def run_psweep(args):
    """Corollary 2 of the paper on the GPU: the agent count that minimises the time to
    a solution.  For each p, the block steps to --tol and the time per step (A.D
    launches timed per step with events, and whole solves) on the --n, --kappa system;
    the time to solution is their product.  The starting columns are the first p of
    one block of 16 (32 when the sweep goes past 16).  One JSON line."""
    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_PROFILE, Context

    dev = "cuda:0"
    n = args.n
    seed = ci.BASE_SEED if args.seed is None else args.seed
    A = ci.spd_spectrum(n, args.kappa, ci.item_seed("A", seed, base=n), device=dev)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", seed, base=n)), device=dev)
    ps = [int(v) for v in args.psweep.split(",") if v]
    pmax = 32 if max(ps) > 16 else 16
    Xall = torch.as_tensor(ci.normal_block(n, pmax, ci.item_seed("X0", seed, base=n)), device=dev)
    ctx = Context(0)
    rows = []
    for p in ps:
        X0 = Xall[:, :p].contiguous()
        ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec)
        torch.cuda.synchronize()
        reps = max(1, args.steps // 5)
        t0 = time.perf_counter()
        for _ in range(reps):
            X, info = ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec)
        torch.cuda.synchronize()
        per_solve = (time.perf_counter() - t0) / reps
        ctx.kernel_time(reset=True)
        ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec, flags=CCG_PROFILE)
        ad_ms, ad_n = ctx.kernel_time(reset=True)
        rows.append({"p": p, "iters": info["iters"], "ms_per_solve": round(per_solve * 1e3, 3),
                     "us_per_step": round(per_solve * 1e6 / max(1, info["iters"]), 2),
                     "ad_us": round(ad_ms * 1e3 / max(1, ad_n), 2), "rel_res": info["rel_res"],
                     "status": info["status_name"]})
        print(json.dumps({"progress": "p", "p": p, "iters": info["iters"]}), file=sys.stderr, flush=True)
    ctx.close()
    best = min(rows, key=lambda r: r["ms_per_solve"])
    print(json.dumps({"mode": "psweep", "workload": f"dense SPD n={n}, kappa={args.kappa:g} (log-uniform "
                                                    f"spectrum), {args.prec.upper()} A, tol {args.tol:g}",
                      "rows": rows, "fastest_p": best["p"],
                      "paper": "Corollary 2 (Sec. 4): the optimal agent count, from the multiplication "
                               "count of Table 1 with A streamed once per agent"}))


def _oracle_rate(samples):
    """Oracle seconds per block step per n^2, from a few (A, b, X0, steps) samples."""
    import oracle
    coef, spent = [], 0.0
    for A, b, X0, k in samples:
        c0 = time.perf_counter()
        oracle.ccg(A, b, X0, tol=0.0, maxit=k)
        dt = time.perf_counter() - c0
        spent += dt
        coef.append(dt / ((k + 1) * A.shape[0] ** 2))
    return float(sum(coef) / len(coef)), spent


def stream_ceiling(args):
    """Read-only streams of an n x n FP64 matrix in the A.D kernel's traffic shape:
    whole columns per workgroup, with and without the per-workgroup re-read of an
    n x p direction block.  One JSON line; GB/s counts the matrix bytes only."""
    import torch  # noqa: F401  (loads the HIP runtime the library shares)
    from paper_1204_0069_amd import Context
    ctx = Context(0)
    n = args.n
    rows = []
    for stagger in (False, True):
        for dcols in (0, args.p):
            for waves in (4, 8, 16):
                for cols in (4, 8, 16, 32):
                    if cols < waves // 2 or cols > 4 * waves:
                        continue
                    us = ctx.stream_probe(n, cols, dcols, stagger=stagger, reps=20, waves=waves)
                    rows.append({"cols_per_workgroup": cols, "waves": waves, "direction_cols": dcols,
                                 "stagger": stagger, "median_us": round(us, 2),
                                 "GB_s": round(8.0 * n * n / (us * 1e-6) / 1e9, 1)})
    # the plain grid-stride read of the same bytes, 1 to 8 workgroups per CU
    for waves in (4, 8, 16):
        for wgs in (256, 512, 1024, 2048):
            if n % wgs:
                continue
            us = ctx.stream_probe(n, n // wgs, 0, stagger=2, reps=20, waves=waves)
            rows.append({"grid_stride_workgroups": wgs, "waves": waves, "median_us": round(us, 2),
                         "GB_s": round(8.0 * n * n / (us * 1e-6) / 1e9, 1)})
    ctx.close()
    print(json.dumps({"probe": "ccg_stream_probe", "n": n, "matrix_bytes": 8 * n * n, "rows": rows}))


def run_batched(args):
    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_ESCALATE, PREC, Context

    dev = "cuda:0"
    specs = ci.batch_specs(count=args.count, n_lo=64, n_hi=4096, p_choices=(2, 4, 8),
                           k_lo=1e2, k_hi=1e5)
    # low-precision systems move to a wider precision when their refinement breaks
    # down (at kappa near 1e5 the BF16x2 copy's rounding times kappa is close to 1)
    flags = CCG_ESCALATE if args.prec != "fp64" else 0
    systems = []
    for sp in specs:
        A = ci.spd_spectrum(sp["n"], sp["kappa"], sp["seed"], device=dev)
        b = torch.as_tensor(ci.normal_block(sp["n"], 0, ci.item_seed("bb", sp["seed"])), device=dev)
        X0 = torch.as_tensor(ci.normal_block(sp["n"], sp["p"], ci.item_seed("bx", sp["seed"])), device=dev)
        systems.append(dict(A=A, b=b, X0=X0, tol=args.tol, maxit=10 ** 6, prec=args.prec, flags=flags))
    torch.cuda.synchronize()
    ctx = Context(0)
    if args.single_fp64:
        return _batched_single_fp64(args, ctx, specs, systems)
    for _ in range(args.warmup):
        ctx.solve_batched(systems[: min(32, len(systems))])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.solve_batched(systems)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    infos = [r[1] for r in res]
    ok = sum(1 for i in infos if i["status"] == 0)
    bytes_a = sum(i["bytes_A"] for i in infos) * args.steps
    eff = bytes_a / total / 1e9
    n2 = np.array([sp["n"] ** 2 for sp in specs], dtype=np.float64)
    cpu = None
    if args.cpu_sample_steps > 0:
        idx = np.argsort(n2)[:: max(1, len(specs) // 6)][:6]
        samples = []
        for i in idx:
            sy = systems[i]
            samples.append((sy["A"].cpu().numpy(), sy["b"].cpu().numpy(), sy["X0"].cpu().numpy(),
                            args.cpu_sample_steps))
        c, spent = _oracle_rate(samples)
        steps_i = np.array([i["iters"] + 2 * (i["refinements"] + 1) for i in infos], dtype=np.float64)
        t_cpu = float(c * (n2 * steps_i).sum())
        cpu = {"value": round(len(specs) / t_cpu, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_sample_steps} FP64 block steps on each of {len(samples)} systems of "
                         f"the batch ({spent:.1f} s); seconds per step per n^2 = {c:.3e}, scaled by "
                         f"sum(n^2 x the GPU's steps per system)"}
    out = {
        "metric": METRIC, "value": round(len(specs) * args.steps / total, 4), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x2": "bf16x2"}[args.prec], "data": "synthetic",
        "config": {"workload": f"batch of {len(specs)} dense SPD systems, n log-uniform in [64, 4096], "
                               f"p in {{2, 4, 8}}, kappa log-uniform in [1e2, 1e5], {args.prec.upper()} A, "
                               f"tol {args.tol:g}"
                               + (", precision escalation on breakdown" if flags else ""),
                   "count": len(specs), "prec": args.prec},
        "converged": ok, "escalated": sum(1 for i in infos if i["prec_final"] != PREC[args.prec]),
        "iters_mean": float(np.mean([i["iters"] for i in infos])),
        "iters_max": int(max(i["iters"] for i in infos)),
        "rel_res_max": float(max(i["rel_res"] for i in infos)),
        "roofline": {"bound": "hbm", "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(eff / HBM_PEAK_GBS, 4), "traffic": None,
                     "kind": "effective: algorithmic A bytes of all systems / wall time"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


def _batched_single_fp64(args, ctx, specs, systems):
    """Plain FP64 baseline of the batched workload: every 8th system of the same batch
    solved with one ccg_solve at a time (no batched engine in the process)."""
    import numpy as np
    import torch
    sample = list(range(0, len(systems), 8))
    for i in sample[: args.warmup]:
        sy = systems[i]
        ctx.solve(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], raise_on_error=False, prec="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in sample:
        sy = systems[i]
        infos.append(ctx.solve(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], raise_on_error=False,
                               prec="fp64")[1])
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    bytes_a = sum(i["bytes_A"] for i in infos)
    eff = bytes_a / total / 1e9
    out = {
        "metric": METRIC, "value": round(len(sample) / total, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": len(sample), "warmup": args.warmup, "ms_per_step": round(total / len(sample) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plain FP64 baseline of the batched workload: every 8th of the batch of "
                               f"{len(specs)} dense SPD systems (n log-uniform in [64, 4096], p in {{2, 4, 8}}, "
                               f"kappa log-uniform in [1e2, 1e5]), one ccg_solve at a time, FP64 A, "
                               f"tol {args.tol:g}", "count": len(sample), "prec": "fp64",
                   "mode": "single-fp64"},
        "converged": sum(1 for i in infos if i["status"] == 0),
        "iters_mean": float(np.mean([i["iters"] for i in infos])),
        "rel_res_max": float(max(i["rel_res"] for i in infos)),
        "roofline": {"bound": "hbm", "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(eff / HBM_PEAK_GBS, 4), "traffic": None,
                     "kind": "effective: algorithmic A bytes of the sampled systems / wall time"},
        "cpu_baseline": None,
    }
    print(json.dumps(out))
    ctx.close()


def run_served(args):
    import numpy as np
    import torch

    import ccg_inputs as ci
    from paper_1204_0069_amd import CCG_ESCALATE, Context

    dev = "cuda:0"
    rng = np.random.default_rng(ci.item_seed("served-pool", ci.BASE_SEED))
    pool = []
    for i in range(args.pool):
        n = int(round(np.exp(rng.uniform(np.log(128), np.log(args.n_hi)))))
        kappa = float(np.exp(rng.uniform(np.log(1e2), np.log(1e6))))
        A = ci.spd_spectrum(n, kappa, ci.item_seed("served-A", i), device=dev)
        pool.append((n, kappa, A.cpu().pin_memory()))
        del A
        if (i + 1) % 8 == 0:
            print(json.dumps({"progress": "pool", "matrices": i + 1}), file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    precs = ("fp64", "fp32", "bf16x2")
    total_req = args.requests + 8
    reqs = []
    for r in range(total_req):
        k = int(rng.integers(0, len(pool)))
        n = pool[k][0]
        b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("served-b", r))).pin_memory()
        X0 = torch.as_tensor(ci.normal_block(n, 4, ci.item_seed("served-x", r))).pin_memory()
        reqs.append((k, b, X0, precs[int(rng.integers(0, 3))]))
    ctx = Context(0, hbm_budget=int(args.budget_gib * (1 << 30)))

    def submit(r):
        k, b, X0, prec = reqs[r]
        # a refinement that breaks down (BF16x2 at the largest condition numbers)
        # continues in FP32, then FP64
        return ctx.submit(pool[k][2], b, X0, args.tol, 10 ** 6, prec=prec, flags=CCG_ESCALATE)

    # warm-up on the first 8 requests, then the timed requests submitted all at once:
    # the service's saturated (closed-loop) rate, which sets the arrival rate
    ts = [submit(r) for r in range(8)]
    for t in ts:
        ctx.wait(t)
    c0 = time.perf_counter()
    ts = [submit(8 + j) for j in range(args.requests)]
    for j, t in enumerate(ts):
        ctx.wait(t)
        if (j + 1) % 200 == 0:
            print(json.dumps({"progress": "closed loop", "requests": j + 1}), file=sys.stderr, flush=True)
    closed = args.requests / (time.perf_counter() - c0)
    rate = args.rate if args.rate > 0 else args.rate_frac * closed
    gaps = rng.exponential(1.0 / rate, args.requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    tickets = []
    t0 = time.perf_counter()
    for j in range(args.requests):
        now = time.perf_counter() - t0
        if arrivals[j] > now:
            time.sleep(arrivals[j] - now)
        tickets.append(submit(8 + j))
        if (j + 1) % 100 == 0:
            print(json.dumps({"progress": "submitted", "requests": j + 1}), file=sys.stderr, flush=True)
    results = []
    for j, t in enumerate(tickets):
        results.append(ctx.wait(t))
        if (j + 1) % 200 == 0:
            print(json.dumps({"progress": "finished", "requests": j + 1}), file=sys.stderr, flush=True)
    total = time.perf_counter() - t0
    infos = [r[1] for r in results]
    lat = np.array([i["seconds"] for i in infos]) * 1e3
    # upload share of each latency: A, b and X0 at the pinned-memory copy rate measured
    # here (largest pool matrix, host to device, after the stream)
    big = max(range(len(pool)), key=lambda k: pool[k][0])
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    tmp = pool[big][2].to(dev, non_blocking=True)
    torch.cuda.synchronize()
    h2d = pool[big][2].numel() * 8 / (time.perf_counter() - u0)
    del tmp
    up_ms = np.array([(pool[reqs[8 + j][0]][0] ** 2 + 5 * pool[reqs[8 + j][0]][0]) * 8 / h2d * 1e3
                      for j in range(args.requests)])
    lat_x = lat - up_ms
    st = {}
    for i, j in zip(infos, range(args.requests)):
        key = f"{reqs[8 + j][3]}:{i['status_name']}"
        st[key] = st.get(key, 0) + 1
    ok = [i for i in infos if i["status"] == 0]
    bytes_a = sum(i["bytes_A"] for i in infos)
    eff = bytes_a / total / 1e9
    out = {
        "metric": METRIC, "value": round(len(ok) / total, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 8, "ms_per_step": round(total / args.requests * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "mixed",
        "data": "synthetic",
        "config": {"workload": f"served stream: Poisson arrivals at {rate:.3f}/s ({rate / closed:.2f} x the "
                               f"closed-loop rate {closed:.3f}/s of the same requests), n log-uniform in "
                               f"[128, {args.n_hi}], p=4, kappa "
                               f"log-uniform in [1e2, 1e6], precision uniform over fp64/fp32/bf16x2, "
                               f"{args.pool} pooled matrices in pinned host memory (upload in latency), "
                               f"precision escalation on breakdown, "
                               f"HBM budget {args.budget_gib:g} GiB", "requests": args.requests},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "latency_ms_excluding_upload": {"p50": round(float(np.percentile(lat_x, 50)), 3),
                                        "p99": round(float(np.percentile(lat_x, 99)), 3),
                                        "h2d_GB_s": round(h2d / 1e9, 1)},
        "statuses": st,
        "rel_res_max_converged": float(max((i["rel_res"] for i in ok), default=float("nan"))),
        "roofline": {"bound": "hbm", "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(eff / HBM_PEAK_GBS, 4), "traffic": None,
                     "kind": "effective: algorithmic A bytes of all requests / wall time"},
        "cpu_baseline": None,
    }
    out["closed_loop_solves_per_s"] = round(closed, 4)
    ctx.close()
    if args.compare_fp64:
        base = Context(0)
        out["plain_fp64"] = _served_fp64_comparison(base, pool, reqs[8:8 + args.requests], arrivals, args, lat)
        service_ms = out["plain_fp64"].pop("service_ms")
        base.close()
    if args.dump:
        recs = [{"n": pool[reqs[8 + j][0]][0], "kappa": pool[reqs[8 + j][0]][1], "prec": reqs[8 + j][3],
                 "arrival_s": float(arrivals[j]), "latency_ms": float(lat[j]), "iters": infos[j]["iters"],
                 "refinements": infos[j]["refinements"], "prec_final": infos[j]["prec_final"],
                 "status": infos[j]["status_name"]} for j in range(args.requests)]
        if args.compare_fp64:
            for r, s_ in zip(recs, service_ms):
                r["fp64_service_ms"] = s_
        with open(args.dump, "w") as f:
            json.dump(recs, f, indent=1)
    print(json.dumps(out))


def _served_fp64_comparison(ctx, pool, reqs, arrivals, args, lat_served):
    """The same requests in plain FP64, one ccg_solve at a time (upload of A from pinned
    host memory included in each service time), and the latencies a first-come
    first-served queue of such solves would give on the same arrival times."""
    import numpy as np
    import torch
    dev = "cuda:0"
    service = []
    ok = 0
    for k, b, X0, _ in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = pool[k][2].to(dev, non_blocking=True)
        _, info = ctx.solve(A, b.to(dev, non_blocking=True), X0.to(dev, non_blocking=True), args.tol, 10 ** 6,
                            raise_on_error=False, prec="fp64")
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        ok += info["status"] == 0
        del A
        if len(service) % 200 == 0:
            print(json.dumps({"progress": "plain fp64", "requests": len(service)}), file=sys.stderr, flush=True)
    finish = 0.0
    lat = []
    for a, s in zip(arrivals, service):
        finish = max(finish, a) + s
        lat.append((finish - a) * 1e3)
    lat = np.array(lat)
    return {"closed_loop_solves_per_s": round(len(service) / sum(service), 4), "converged": int(ok),
            "service_ms": [round(x * 1e3, 3) for x in service],
            "fifo_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                "p99": round(float(np.percentile(lat, 99)), 3)},
            "fifo_note": "first-come first-served queue of one-at-a-time FP64 solves on the served "
                         "stream's arrival times, from each request's measured FP64 service time",
            "fifo_p50_over_served_p50": round(float(np.percentile(lat, 50) / np.percentile(lat_served, 50)), 3),
            "fifo_p99_over_served_p99": round(float(np.percentile(lat, 99) / np.percentile(lat_served, 99)), 3)}


if __name__ == "__main__":
    main()
