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
    ap.add_argument("--mode", default="single", choices=["single", "batched", "served"])
    ap.add_argument("--kind", default="spectrum", choices=["spectrum", "gram"],
                    help="single mode: Q diag(lam) Q^T, or M^T M / n + sigma I")
    ap.add_argument("--count", type=int, default=1024, help="batched mode: systems per batch")
    ap.add_argument("--requests", type=int, default=48, help="served mode: timed requests")
    ap.add_argument("--pool", type=int, default=12, help="served mode: distinct matrices")
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
    infos = []
    for _ in range(args.warmup):
        ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec, flags=flags)
    ctx.kernel_time(reset=True)

    # Timed region: the A.D launches of every 4th round of block steps bracketed by
    # HIP events on the library's stream (launched directly); the other rounds replay
    # the captured graph (CCG_PROFILE_SAMPLED; --profile-all times every launch).
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        X, info = ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec, flags=flags)
        lat.append(time.perf_counter() - s0)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = t1 - t0
    ad_ms, ad_launches = ctx.kernel_time(reset=True)

    # Second region, same solves through captured graphs and no events (context only).
    graph_rate = None
    if not args.no_profile:
        ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve(A, b, X0, args.tol, 100000, prec=args.prec)
        torch.cuda.synchronize()
        graph_rate = args.steps / (time.perf_counter() - g0)

    iters = [i["iters"] for i in infos]
    # explicit residual of the last result, independent of the library (rocBLAS)
    T = b[:, None] - A @ X
    rel = (torch.linalg.norm(T, dim=0) / torch.linalg.norm(b)).cpu().numpy()

    s_a = {"fp64": 8, "fp32": 4, "bf16x2": 4}[args.prec]
    s_v = 8 if args.prec == "fp64" else 4
    bytes_per_launch = n * n * s_a + 2 * n * p * s_v
    roofline = None
    if ad_launches > 0:
        avg_s = ad_ms / 1e3 / ad_launches
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": recorded_traffic(n, p, args.prec), "traffic_unit": "B/launch",
                    "kernel": "k_ad",
                    "avg_launch_us": round(avg_s * 1e6, 2), "launches": ad_launches,
                    "timed": ("every A.D launch" if args.profile_all else
                              "the A.D launches of every 4th round of block steps"),
                    "bytes_per_launch": bytes_per_launch}

    cpu = None
    if args.cpu_sample_steps > 0:
        import oracle
        An = A.cpu().numpy()
        bn = b.cpu().numpy()
        Xn = X0.cpu().numpy()
        c0 = time.perf_counter()
        oracle.ccg(An, bn, Xn, tol=0.0, maxit=args.cpu_sample_steps)
        c1 = time.perf_counter()
        per_step = (c1 - c0) / (args.cpu_sample_steps + 1)   # + the initial residual pass
        steps_per_solve = float(np.mean(iters)) + 2.0        # + initial and confirming residuals
        cpu = {"value": round(1.0 / (per_step * steps_per_solve), 6), "unit": "solves/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_sample_steps} block steps of the same n={n}, p={p} system "
                         f"({c1 - c0:.1f} s, {per_step:.3f} s per A stream); solves/s = 1 / "
                         f"(s per step x {steps_per_solve:.0f} steps per solve)"}

    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": round(args.steps / total, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3),
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
        "solves_per_s_graph": None if graph_rate is None else round(graph_rate, 4),
        "iters_per_solve": float(np.mean(iters)),
        "restarts": int(sum(i["restarts"] for i in infos)),
        "rel_res": float(rel.min()),
        "status": infos[-1]["status_name"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


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

    # closed loop on the first 8 requests: saturated rate (and warm-up)
    c0 = time.perf_counter()
    ts = [submit(r) for r in range(8)]
    for t in ts:
        ctx.wait(t)
    closed = 8 / (time.perf_counter() - c0)
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
    results = [ctx.wait(t) for t in tickets]
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
                               f"closed-loop rate {closed:.3f}/s of the first 8 requests), n log-uniform in "
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
    if args.compare_fp64:
        # the same requests submitted all at once: the service's saturated rate
        c0 = time.perf_counter()
        ts = [submit(8 + j) for j in range(args.requests)]
        for t in ts:
            ctx.wait(t)
        out["closed_loop_solves_per_s"] = round(args.requests / (time.perf_counter() - c0), 4)
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
