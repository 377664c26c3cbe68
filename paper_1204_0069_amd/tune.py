"""Autotuner of the A.D tile shape (A columns per wave, waves per workgroup) on the GPU.

    python -m paper_1204_0069_amd.tune [--reps 10] [--out csrc/ccg_tune_table.h]

For every precision, padded agent count P and a ladder of system sizes n it times
the full A.D launch of the block step (stream of A, Gram products, stop test and
p x p solves) for each candidate shape with ccg_tune_ad, in the single-system kernel
and in the batched one (a system solved batched uses the shape its single solve
uses, so that both give the same result; the batched kernel needs more registers
and spills in some shapes), scores each shape by the slower of the two, keeps the
best, merges neighbouring sizes with the same choice into n ranges and writes the
table that the library compiles in (csrc/ccg_tune_table.h).  Rebuild the library
afterwards (python -m paper_1204_0069_amd.build).

The shape changes the tile decomposition, hence the order in which the Gram
partial sums are added; the table is fixed at build time, so results stay
reproducible from run to run.
"""
from __future__ import annotations

import argparse
import datetime
import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "csrc", "ccg_tune_table.h")

PRECS = (("fp64", "PREC_F64"), ("fp32", "PREC_F32"), ("bf16x2", "PREC_BF16X2"))
AGENTS = (1, 2, 4, 8, 16)      # (32: FP64 only, timed with --agents 32 --prec fp64)
SIZES = (128, 256, 512, 1024, 2048, 4096, 8192, 16384)
WIDTHS = (1, 2, 4)
WAVES = (4, 8, 16)
DEFAULT = (2, 4)


def fits4(prec: str, P: int) -> bool:
    """Mirror of the library's rule for 4 columns per wave (ad_cw4_fits)."""
    return P < 16 and (prec != "fp64" or P <= 4)


# Padded agent counts whose shapes may use more than 4 waves per workgroup.  At P <= 4
# the wider shapes won in the one-system timings but lost in the engine, which runs
# several systems of a class in one launch: the served stream (p = 4) fell from 18.0
# to 16.6 requests/s with them, on one box.
WIDE_P = (8,)


# Shapes that run the matrix-core tiles (ad_has_mfma, ad_cw_fit): 16 or 32 rows per
# workgroup (cw * nw), nw waves splitting the contraction.  FP64 at P = 8, 16 and 32;
# FP32 and BF16x2 (FP32 operands) at P = 16.
MFMA_SHAPES = {8: ((4, 4), (4, 8)), 16: ((4, 4), (2, 8), (4, 8), (1, 16), (2, 16)),
               32: ((4, 4), (2, 8), (4, 8), (1, 16), (2, 16))}


def shapes(prec: str, P: int):
    """Candidate (columns per wave, waves per workgroup), as the library runs them
    (ad_cw_fit, ad_nw_fit): vector tiles with 4 columns where they fit and more than
    4 waves at WIDE_P, then the matrix-core shapes."""
    if P == 32:                # the matrix-core tile only (FP64)
        return list(MFMA_SHAPES[32]) if prec == "fp64" else []
    ws = [w for w in WIDTHS if w < 4 or fits4(prec, P)]
    if P >= 16:
        ws = [w for w in ws if w <= 2]
    nws = WAVES if P in WIDE_P else (4,)
    out = [(w, nw) for nw in nws for w in ws]
    if prec == "fp64" or P == 16:
        out += [sh for sh in MFMA_SHAPES.get(P, ()) if sh not in out]
    return out


MARGIN = 0.03   # another shape must beat the default (2, 4) by 3 % to be chosen


def choose(t: dict):
    """Fastest shape, keeping the default unless another is clearly faster (short
    launches differ by timing noise)."""
    w = min(t, key=t.get)
    if DEFAULT in t and t[DEFAULT] <= (1.0 + MARGIN) * t[w]:
        return DEFAULT
    return w


def rows_from(best_by_class):
    """Table rows from {(cname, P): [(n, shape), ...]}: neighbouring sizes with the
    same shape merge, and a row covers sizes up to 1.5 x its largest timed n."""
    rows = []
    for (cname, P), best in best_by_class.items():
        merged = []
        for n, w in best:
            if merged and merged[-1][1] == w:
                merged[-1] = (n, w)
            else:
                merged.append((n, w))
        for i, (n, w) in enumerate(merged):
            last = i == len(merged) - 1
            rows.append((cname, P, (1 << 30) if last else n + (n // 2), w[0], w[1]))
    return rows


def tune(ctx, reps: int, log=print, precs=None, agents=AGENTS, sizes=SIZES):
    best_by_class = {}
    for prec, cname in PRECS:
        if precs and prec not in precs:
            continue
        for P in agents:
            best = []
            for n in sizes:
                if P > n:
                    continue
                ts = {sh: ctx.tune_ad(prec, P, n, sh[0], reps, nw=sh[1]) for sh in shapes(prec, P)}
                tb = {sh: ctx.tune_ad(prec, P, n, sh[0], reps, nw=sh[1], batched=True) for sh in shapes(prec, P)}
                t = {sh: max(ts[sh], tb[sh]) for sh in ts}
                sh = choose(t)
                best.append((n, sh))
                log(f"{prec:7s} P={P:2d} n={n:6d} "
                    + "  ".join(f"c{k[0]}w{k[1]}:{v:9.2f}us({ts[k]:.2f}/{tb[k]:.2f})" for k, v in t.items())
                    + f"  -> {sh[0]},{sh[1]}")
            best_by_class[(cname, P)] = best
    return rows_from(best_by_class)


def rows_from_log(path: str):
    """Re-tabulate the timings a previous run printed (no GPU needed)."""
    import re
    names = dict(PRECS)
    best_by_class = {}
    for line in open(path):
        m = re.match(r"(\w+)\s+P=\s*(\d+) n=\s*(\d+) (.*)  -> \d", line)
        if not m:
            continue
        prec, P, n = m.group(1), int(m.group(2)), int(m.group(3))
        # "c2w8: 91.3us(90.1/91.3)" entries (the score, then the single-system and the
        # batched time), or "cw2: 91.3us" from logs of 4-wave workgroups only
        t = {(int(c), int(w)): float(v) for c, w, v in re.findall(r"c(\d)w(\d+):\s*([\d.]+)us", m.group(4))}
        t.update({(int(c), 4): float(v) for c, v in re.findall(r"cw(\d):\s*([\d.]+)us", m.group(4))})
        allowed = set(shapes(prec, P))
        t = {k: v for k, v in t.items() if k in allowed}
        best_by_class.setdefault((names[prec], P), []).append((n, choose(t)))
    return rows_from(best_by_class)


def write_table(rows, device: str, path: str = OUT):
    lines = [
        "// A.D tile shapes (A columns per wave, waves per workgroup) by precision, padded",
        "// agent count and system size.  Written by `python -m paper_1204_0069_amd.tune`",
        "// from timings of every candidate shape on the GPU; the first row whose (prec, P)",
        "// match and whose n_max >= n applies, and a size no row covers uses 2 and 4.",
        f"// Tuned on: {device}, {datetime.date.today().isoformat()}.",
        "#pragma once",
        "",
        "namespace ccg {",
        "",
        "struct TuneRow {",
        "    int prec;     // Prec",
        "    int P;        // padded agent count",
        "    int n_max;    // largest n of the row",
        "    int cw;       // A columns per wave: 1, 2 or 4",
        "    int nw;       // waves per workgroup: 4, 8 or 16",
        "};",
        "",
        "static const TuneRow kTuneTable[] = {",
    ]
    lines += [f"    {{{c}, {P}, {n_max}, {w}, {nw}}}," for c, P, n_max, w, nw in rows]
    lines += ["};", "", "}  // namespace ccg", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--from-log", default=None, help="re-tabulate a saved tuner log")
    ap.add_argument("--device", default="AMD Instinct MI355X", help="device name for --from-log")
    ap.add_argument("--prec", default=None, help="comma-separated precisions to time (default: all)")
    ap.add_argument("--agents", default=None, help="comma-separated padded agent counts (default: all)")
    ap.add_argument("--sizes", default=None, help="comma-separated n (default: the full ladder)")
    ap.add_argument("--no-write", action="store_true", help="print the timings only")
    args = ap.parse_args()
    if args.from_log:
        rows = rows_from_log(args.from_log)
        write_table(rows, args.device + " (timings of " + os.path.basename(args.from_log) + ")", args.out)
        print(f"wrote {len(rows)} rows to {args.out}")
        return
    import torch
    from .ccg import Context
    ctx = Context(0)
    precs = args.prec.split(",") if args.prec else None
    agents = tuple(int(v) for v in args.agents.split(",")) if args.agents else AGENTS
    sizes = tuple(int(v) for v in args.sizes.split(",")) if args.sizes else SIZES
    rows = tune(ctx, args.reps, log=lambda s: print(s, flush=True), precs=precs, agents=agents, sizes=sizes)
    if not args.no_write:
        write_table(rows, torch.cuda.get_device_name(0), args.out)
        print(f"wrote {len(rows)} rows to {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()
