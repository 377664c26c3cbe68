"""Every A.D tile width the tuned table selects gives oracle-matching steps.

The table (csrc/ccg_tune_table.h) picks 1, 2 or 4 A columns per wave by precision,
agent count and n; each width is a separate kernel instantiation.  For every
(precision, P) class below and every width the table uses for it, a system whose n
falls in that row runs through the library: FP64 block steps against the oracle
(per step, 1e-10), FP32 refined solves against the explicit FP64 residual.
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
    rows = [(c, int(P), int(n), int(w)) for c, P, n, w in
            re.findall(r"\{(PREC_\w+), (\d+), (\d+), (\d)\}", open(TABLE).read())]
    out = []
    for P in Ps:
        lo = 0
        seen = set()
        for c, PP, n_max, w in rows:
            if c != prec_name or PP != P:
                continue
            n = max(lo + 1, 64, P)
            if w not in seen and n <= min(n_max, n_cap):
                out.append((P, n, w))
                seen.add(w)
            lo = n_max
    return out


FP64_CASES = _cases("PREC_F64", (1, 4, 8), 4096)
FP32_CASES = _cases("PREC_F32", (2, 8), 4096)


@pytest.mark.parametrize("P,n,w", FP64_CASES)
def test_fp64_steps_at_each_width(gpu_ctx, P, n, w):
    p = max(1, P - 1) if P > 1 else 1
    print(f"case width {w} fp64 n={n} p={p}", flush=True)
    A, b, X0 = ci.system(n, p, 1e3, seed=1300 + n)
    k = 4
    orc = oracle.ccg(A, b, X0, tol=0.0, maxit=k, trace_k=k, want_rd=True)
    g = gpu_ctx.debug_step(_t(A), _t(b), _t(X0), k)
    for s in range(k):
        assert np.abs(g["alphas"][s] - orc["alphas"][s]).max() <= 1e-10 * np.abs(orc["alphas"][s]).max()
        assert np.abs(g["betas"][s] - orc["betas"][s]).max() <= 1e-10 * np.abs(orc["betas"][s]).max()
    Xg = g["X"].numpy()
    assert np.linalg.norm(Xg - orc["X"]) <= 1e-10 * np.linalg.norm(orc["X"])


@pytest.mark.parametrize("P,n,w", FP32_CASES)
def test_fp32_solve_at_each_width(gpu_ctx, P, n, w):
    p = P
    print(f"case width {w} fp32 n={n} p={p}", flush=True)
    A, b, X0 = ci.system(n, p, 1e2, seed=1400 + n)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32")
    assert info["status"] == 0, info
    T = oracle.residual(A, b, X.cpu().numpy())
    assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= 1.01e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_tuner_entry_times_every_width(gpu_ctx, prec):
    for w in (1, 2, 4):
        us = gpu_ctx.tune_ad(prec, 4, 512, w, reps=2)
        assert 0.0 < us < 1e5


def test_stream_probe_times_the_traffic_shape(gpu_ctx):
    """The read-only floor probe runs in every shape bench.py asks of it and reports a
    positive time; re-reading the direction block does not make it faster."""
    t0 = gpu_ctx.stream_probe(1024, 8, 0, stagger=False, reps=3)
    t1 = gpu_ctx.stream_probe(1024, 8, 8, stagger=True, reps=3)
    assert 0.0 < t0 < 1e5 and 0.0 < t1 < 1e5
    assert t1 >= 0.5 * t0
    with pytest.raises(Exception):
        gpu_ctx.stream_probe(1000, 3, 0)          # cols must divide n
