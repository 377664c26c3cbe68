"""Every A.D tile width the tuned table selects gives oracle-matching steps.

The table (csrc/ccg_tune_table.h) picks 1, 2 or 4 A columns per wave and 4, 8 or 16
waves per workgroup by precision, agent count and n; each shape is a separate kernel
instantiation.  For every
(precision, P) class below and every width the table uses for it, a system whose n
falls in that row runs through the library: FP64 block steps against the oracle
(per step, 1e-10), FP32 and BF16 hi+lo refined solves against the explicit FP64 residual.
"""
import os
import re

import numpy as np
import pytest
import torch

import ccg_inputs as ci
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TABLE = os.path.join(os.path.dirname(__file__), "..", "paper_1204_0069_amd", "csrc", "ccg_tune_table.h")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _cases(prec_name, Ps, n_cap):
    """One (P, n, width, waves) case per tile shape the table uses for each P, at the
    smallest n of the first row that selects it, and at least 8 P (4 steps of p = 15
    agents at n = 64 come within a step of finite termination, where the FP64 oracle
    itself drifts 3e-10 from an extended-precision run); sizes above n_cap are
    skipped."""
    rows = [(c, int(P), int(n), int(w), int(nw)) for c, P, n, w, nw in
            re.findall(r"\{(PREC_\w+), (\d+), (\d+), (\d), (\d+)\}", open(TABLE).read())]
    out = []
    for P in Ps:
        lo = 0
        seen = set()
        for c, PP, n_max, w, nw in rows:
            if c != prec_name or PP != P:
                continue
            n = max(lo + 1, 64, 8 * P)
            if (w, nw) not in seen and n <= min(n_max, n_cap):
                out.append((P, n, w, nw))
                seen.add((w, nw))
            lo = n_max
    return out


def _system(n, p, kappa, seed):
    """Spectrum systems up to n = 4096; larger ones use the Gram construction built on
    the device (a QR of that size on the host takes too long for a test)."""
    if n <= 4096:
        return ci.system(n, p, kappa, seed=seed)
    A, b, X0 = ci.system(n, p, kappa, seed=seed, device=DEV, kind="gram")
    return A.cpu().numpy(), b, X0


FP64_CASES = _cases("PREC_F64", (1, 4, 8, 16), 8192)
FP32_CASES = _cases("PREC_F32", (2, 8, 16), 8192)
LOW_CASES = [("fp32",) + c for c in FP32_CASES] + [("bf16x2",) + c for c in _cases("PREC_BF16X2", (4, 8, 16), 8192)]


@pytest.mark.parametrize("P,n,w,nw", FP64_CASES)
def test_fp64_steps_at_each_width(gpu_ctx, P, n, w, nw):
    p = max(1, P - 1) if P > 1 else 1
    print(f"case width {w} waves {nw} fp64 n={n} p={p}", flush=True)
    A, b, X0 = _system(n, p, 1e3, 1300 + n)
    k = 4
    orc = oracle.ccg(A, b, X0, tol=0.0, maxit=k, trace_k=k, want_rd=True)
    g = gpu_ctx.debug_step(_t(A), _t(b), _t(X0), k)
    for s in range(k):
        assert np.abs(g["alphas"][s] - orc["alphas"][s]).max() <= 1e-10 * np.abs(orc["alphas"][s]).max()
        assert np.abs(g["betas"][s] - orc["betas"][s]).max() <= 1e-10 * np.abs(orc["betas"][s]).max()
    Xg = g["X"].numpy()
    assert np.linalg.norm(Xg - orc["X"]) <= 1e-10 * np.linalg.norm(orc["X"])


@pytest.mark.parametrize("prec,P,n,w,nw", LOW_CASES)
def test_refined_solve_at_each_width(gpu_ctx, prec, P, n, w, nw):
    p = P
    print(f"case width {w} waves {nw} {prec} n={n} p={p}", flush=True)
    A, b, X0 = _system(n, p, 1e2, 1400 + n)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec=prec)
    assert info["status"] == 0, info
    T = oracle.residual(A, b, X.cpu().numpy())
    assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= 1.01e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_tuner_entry_times_every_width(gpu_ctx, prec):
    for w in (1, 2, 4):
        for nw in (4, 8, 16):
            for batched in (False, True):
                us = gpu_ctx.tune_ad(prec, 4, 515, w, reps=2, nw=nw, batched=batched)
                assert 0.0 < us < 1e5
    with pytest.raises(Exception):
        gpu_ctx.tune_ad(prec, 4, 512, 2, reps=2, nw=6)


def test_stream_probe_times_the_traffic_shape(gpu_ctx):
    """The read-only floor probe runs in every shape bench.py asks of it and reports a
    positive time; re-reading the direction block does not make it faster."""
    for waves in (4, 8, 16):
        t0 = gpu_ctx.stream_probe(1024, 8, 0, stagger=False, reps=3, waves=waves)
        t1 = gpu_ctx.stream_probe(1024, 8, 8, stagger=True, reps=3, waves=waves)
        assert 0.0 < t0 < 1e5 and 0.0 < t1 < 1e5
        assert t1 >= 0.5 * t0
        t2 = gpu_ctx.stream_probe(1024, 8, 0, stagger=2, reps=3, waves=waves)   # grid-stride
        assert 0.0 < t2 < 1e5
    with pytest.raises(Exception):
        gpu_ctx.stream_probe(1000, 3, 0)          # cols must divide n
    with pytest.raises(Exception):
        gpu_ctx.stream_probe(1024, 8, 8, stagger=2)   # the grid-stride read has no D
    with pytest.raises(Exception):
        gpu_ctx.stream_probe(1024, 8, 0, waves=6)
