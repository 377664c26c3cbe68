"""GPU tests of the multi-system engine: ccg_solve_batched and the served mode
(ccg_submit / ccg_poll / ccg_wait / ccg_cancel).

The engine runs every system through the same kernels, tile decomposition and phase
sequence as a single ccg_solve, only sharing launches with other systems, so each
system's result must be bit-identical to its single solve (which the parity tests
hold against the oracle); a few systems are also checked against the oracle
directly.
"""
import numpy as np
import pytest
import torch

import ccg_inputs as ci
import oracle
from paper_1204_0069_amd import Context

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


MIXED = [  # n, p, kappa, prec
    (64, 2, 1e2, "fp64"), (256, 3, 1e3, "fp64"), (777, 2, 1e2, "fp64"), (1000, 5, 1e3, "fp64"),
    (129, 4, 10.0, "fp64"), (640, 16, 1e2, "fp64"), (300, 1, 1e3, "fp64"), (2085, 8, 1e4, "fp64"),
    (500, 4, 1e3, "fp32"), (96, 2, 1e2, "fp32"), (1100, 8, 1e3, "fp32"), (900, 12, 1e2, "fp32"),
    (400, 3, 1e2, "bf16x2"), (700, 8, 1e3, "bf16x2"), (600, 14, 1e2, "bf16x2"),
]


def _systems(cases, seed=500, tol=1e-10, maxit=20000):
    out = []
    for i, (n, p, kappa, prec) in enumerate(cases):
        A, b, X0 = ci.system(n, p, kappa, seed=seed + i)
        out.append(dict(A=_t(A), b=_t(b), X0=_t(X0), tol=tol, maxit=maxit, prec=prec))
    return out


def _single(ctx, sy):
    opts = {k: v for k, v in sy.items() if k not in ("A", "b", "X0", "tol", "maxit")}
    return ctx.solve(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], raise_on_error=False, **opts)


def _same(a, b):
    (Xa, ia), (Xb, ib) = a, b
    assert ia["status"] == ib["status"], (ia, ib)
    for f in ("iters", "refinements", "restarts", "deflations", "p_final", "best_agent"):
        assert ia[f] == ib[f], (f, ia, ib)
    assert ia["rel_res"] == ib["rel_res"]
    assert torch.equal(Xa, Xb)


def test_batched_equals_single_solves(gpu_ctx):
    print(f"case batched mixed {len(MIXED)} systems", flush=True)
    systems = _systems(MIXED)
    singles = [_single(gpu_ctx, sy) for sy in systems]
    batched = gpu_ctx.solve_batched(systems)
    for s, b in zip(singles, batched):
        _same(s, b)
    assert all(b[1]["status"] == 0 for b in batched)


def test_batched_against_oracle(gpu_ctx):
    cases = [(256, 3, 1e3, "fp64"), (1000, 4, 1e3, "fp64"), (513, 2, 1e2, "fp64")]
    systems = _systems(cases, seed=700, tol=1e-11)
    res = gpu_ctx.solve_batched(systems)
    for sy, (X, info) in zip(systems, res):
        A, b, X0 = (sy[k].cpu().numpy() for k in ("A", "b", "X0"))
        assert info["status"] == 0
        same = oracle.ccg(A, b, X0, tol=0.0, maxit=info["iters"])
        Xg = X.cpu().numpy()
        for j in range(Xg.shape[1]):
            assert np.linalg.norm(Xg[:, j] - same["X"][:, j]) <= 1e-10 * np.linalg.norm(same["X"][:, j])


def test_batched_under_a_small_budget(gpu_ctx):
    """A budget that holds two FP32 copies of A at a time: the rest wait for memory."""
    systems = _systems([(2048, 4, 1e3, "fp32")] * 4 + [(700, 4, 1e3, "fp64")], seed=800)
    ref = gpu_ctx.solve_batched(systems)
    ctx = Context(0, hbm_budget=40 << 20)
    try:
        res = ctx.solve_batched(systems)
    finally:
        ctx.close()
    for a, b in zip(ref, res):
        _same(a, b)


def test_batched_system_over_budget_gets_nomem(gpu_ctx):
    # the FP32 copy of a 3000 x 3000 matrix alone (36 MB) exceeds the budget
    systems = _systems([(256, 3, 1e3, "fp64"), (3000, 4, 1e3, "fp32"), (200, 2, 1e2, "fp64")], seed=900)
    ctx = Context(0, hbm_budget=16 << 20)
    try:
        res = ctx.solve_batched(systems)
    finally:
        ctx.close()
    assert [r[1]["status"] for r in res] == [0, -5, 0]


def test_batched_host_pointers_and_bad_problem(gpu_ctx):
    systems = _systems([(300, 3, 1e3, "fp64"), (500, 2, 1e2, "fp32")], seed=950)
    ref = gpu_ctx.solve_batched(systems)
    host = [dict(sy, A=sy["A"].cpu(), b=sy["b"].cpu(), X0=sy["X0"].cpu()) for sy in systems]
    bad = dict(systems[0], tol=-1.0)
    res = gpu_ctx.solve_batched(host + [bad])
    for a, b in zip(ref, res[:2]):
        assert a[1]["iters"] == b[1]["iters"]
        assert torch.equal(a[0].cpu(), b[0])
    assert res[2][1]["status"] == -1


def test_batched_workload_of_many_sizes(gpu_ctx):
    """Sizes, agent counts and condition numbers drawn like the many-system workload
    (n log-uniform, p in {2, 4, 8}, kappa log-uniform), FP32 with FP64 refinement."""
    specs = ci.batch_specs(count=40, n_lo=64, n_hi=1024, k_lo=1e2, k_hi=1e4)
    systems, mats = [], []
    for sp in specs:
        A, b, X0 = ci.system(sp["n"], sp["p"], sp["kappa"], seed=sp["seed"])
        mats.append((A, b))
        systems.append(dict(A=_t(A), b=_t(b), X0=_t(X0), tol=1e-10, maxit=50000, prec="fp32"))
    res = gpu_ctx.solve_batched(systems)
    for (A, b), (X, info) in zip(mats, res):
        assert info["status"] == 0, info
        T = oracle.residual(A, b, X.cpu().numpy())
        rel = np.linalg.norm(T, axis=0) / np.linalg.norm(b)
        assert rel.min() <= 1e-10 * 1.01


# ---------------------------------------------------------------- served mode

def test_served_equals_single_solves(gpu_ctx):
    print(f"case served {len(MIXED)} systems", flush=True)
    systems = _systems(MIXED, seed=1000)
    singles = [_single(gpu_ctx, sy) for sy in systems]
    ctx = Context(0)
    try:
        tickets = [ctx.submit(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], prec=sy["prec"])
                   for sy in systems]
        outs = [ctx.wait(t) for t in tickets]
        for s, o in zip(singles, outs):
            _same(s, o)
            assert o[1]["seconds"] > 0.0
    finally:
        ctx.close()


def test_served_budget_poll_cancel_and_host_pointers(gpu_ctx):
    ctx = Context(0, hbm_budget=40 << 20)
    try:
        systems = _systems([(2048, 4, 1e3, "fp32")] * 3 + [(1024, 4, 1e3, "fp64")], seed=1100)
        ref = [_single(gpu_ctx, sy) for sy in systems]
        # a system that cannot converge (tolerance below rounding) runs until cancelled
        A, b, X0 = ci.system(1500, 4, 1e3, seed=1200)
        long_t = ctx.submit(_t(A), _t(b), _t(X0), 1e-30, 10 ** 7)
        tickets = [ctx.submit(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], prec=sy["prec"])
                   for sy in systems]
        host = systems[3]
        ht = ctx.submit(host["A"].cpu().pin_memory(), host["b"].cpu().pin_memory(),
                        host["X0"].cpu().pin_memory(), host["tol"], host["maxit"])
        outs = [ctx.wait(t) for t in tickets]
        for s, o in zip(ref, outs):
            _same(s, o)
        Xh, ih = ctx.wait(ht)
        assert ih["iters"] == ref[3][1]["iters"] and torch.equal(Xh, ref[3][0].cpu())
        assert ctx.poll(long_t) is None           # still running
        ctx.cancel(long_t)
        X, info = ctx.wait(long_t)
        assert info["status"] == -8 and info["iters"] > 0
        with pytest.raises(Exception):
            ctx.poll(123456789)
    finally:
        ctx.close()


def test_batched_escalation_equals_single(gpu_ctx):
    from paper_1204_0069_amd import CCG_ESCALATE
    systems = _systems([(128, 4, 1e8, "bf16x2"), (300, 3, 1e5, "bf16x2"), (200, 2, 1e2, "fp32")],
                       seed=1500, tol=1e-5, maxit=100000)
    for sy in systems:
        sy["flags"] = CCG_ESCALATE
    singles = [_single(gpu_ctx, sy) for sy in systems]
    batched = gpu_ctx.solve_batched(systems)
    for s, b in zip(singles, batched):
        _same(s, b)
        assert s[1]["prec_final"] == b[1]["prec_final"]
    assert all(b[1]["status"] == 0 for b in batched), [b[1] for b in batched]
    assert batched[0][1]["prec_final"] != 2      # the first system escalated

# Systems with n >= 4096 run in the large-system lane (its own stream and thread),
# the rest in the small-system lane; the lanes share the context's HBM budget.
LANES = [(4096, 2, 1e2, "fp64"), (4200, 4, 1e2, "fp32"), (4200, 3, 1e2, "fp32"),
         (300, 3, 1e3, "fp64"), (900, 4, 1e3, "fp32"), (1500, 2, 1e2, "bf16x2")]


def test_both_lanes_equal_single_solves_under_a_shared_budget(gpu_ctx):
    """The two FP32 copies of the n = 4200 matrices (70 MB each) do not fit the 100 MB
    budget together, so the large lane runs them one after the other while the small
    lane goes on; every result equals its single solve, batched and served."""
    print("case lanes: batched and served, 6 systems, budget 100 MB", flush=True)
    systems = _systems(LANES, seed=1600)
    singles = [_single(gpu_ctx, sy) for sy in systems]
    ctx = Context(0, hbm_budget=100 << 20)
    try:
        batched = ctx.solve_batched(systems)
        tickets = [ctx.submit(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], prec=sy["prec"])
                   for sy in systems]
        served = [ctx.wait(t) for t in tickets]
    finally:
        ctx.close()
    for s_, b_, v_ in zip(singles, batched, served):
        _same(s_, b_)
        _same(s_, v_)
    assert all(b_[1]["status"] == 0 for b_ in batched)


def test_served_mix_with_a_poisoned_request(gpu_ctx):
    """One request in a served mix has a NaN in b.  It ends with CCG_ERR_NONFINITE
    (its first residual norm is not finite) and leaves the service running; every
    other request, submitted before and after it, still equals its single solve."""
    print("case served mix with a NaN right-hand side", flush=True)
    systems = _systems([(300, 3, 1e3, "fp64"), (500, 4, 1e3, "fp32"), (900, 2, 1e2, "bf16x2"),
                        (4100, 2, 1e2, "fp64"), (700, 8, 1e3, "fp64")], seed=1700)
    singles = [_single(gpu_ctx, sy) for sy in systems]
    bad = dict(systems[0])
    bb = bad["b"].clone()
    bb[17] = float("nan")
    bad["b"] = bb
    ctx = Context(0)
    try:
        t = [ctx.submit(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], prec=sy["prec"])
             for sy in systems[:2]]
        tb = ctx.submit(bad["A"], bad["b"], bad["X0"], bad["tol"], bad["maxit"], prec=bad["prec"])
        t += [ctx.submit(sy["A"], sy["b"], sy["X0"], sy["tol"], sy["maxit"], prec=sy["prec"])
              for sy in systems[2:]]
        outs = [ctx.wait(x) for x in t]
        Xb, ib = ctx.wait(tb)
        for s, o in zip(singles, outs):
            _same(s, o)
        assert ib["status"] == -2, ib
        # the service still takes requests
        again = ctx.wait(ctx.submit(systems[4]["A"], systems[4]["b"], systems[4]["X0"], 1e-10, 20000))
        _same(singles[4], again)
    finally:
        ctx.close()
