"""The symmetric A.D pass (CCG_SYM_AD: FP64 block steps of systems with n >= 1024 and
p <= 8 read only the upper block triangle of A, 128 x 128 blocks, and add the partial
sums in a fixed order) against the oracle, and against the whole-matrix kernel."""
import numpy as np
import pytest
import torch

import ccg_inputs as ci
import oracle
from paper_1204_0069_amd import CCG_PROFILE, CCG_SYM_AD, Context

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# n: whole blocks, a ragged last block (one row, odd, most of a block), strips of
# fewer than four blocks; p: every padded agent count of the pass
STEP_CASES = [(1024, 1), (1024, 2), (1025, 3), (1100, 4), (1279, 5), (1536, 8), (2047, 7), (3000, 8)]


@pytest.mark.parametrize("n,p", STEP_CASES)
def test_symmetric_steps_match_oracle(gpu_ctx, n, p):
    print(f"case symmetric debug_step n={n} p={p}", flush=True)
    A, b, X0 = ci.system(n, p, 1e3, seed=2200 + n + p)
    k = 4
    orc = oracle.ccg(A, b, X0, tol=0.0, maxit=k, trace_k=k, want_rd=True)
    g = gpu_ctx.debug_step(_t(A), _t(b), _t(X0), k, flags=CCG_SYM_AD)
    for s in range(k):
        assert np.abs(g["alphas"][s] - orc["alphas"][s]).max() <= 1e-10 * np.abs(orc["alphas"][s]).max()
        assert np.abs(g["betas"][s] - orc["betas"][s]).max() <= 1e-10 * np.abs(orc["betas"][s]).max()
    for key in ("X", "R", "D"):
        assert _rel(g[key].numpy(), orc[key]) <= 1e-10, key


def test_symmetric_and_whole_matrix_solves_agree(gpu_ctx):
    n, p = 2300, 6
    print(f"case symmetric vs whole-matrix solve n={n} p={p}", flush=True)
    A, b, X0 = ci.system(n, p, 1e3, seed=2301)
    Xs, i_s = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=CCG_SYM_AD)
    Xf, i_f = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000)
    assert i_s["status"] == 0 and i_f["status"] == 0
    assert abs(i_s["iters"] - i_f["iters"]) <= max(3, 0.05 * i_f["iters"])
    for X in (Xs, Xf):
        T = oracle.residual(A, b, X.cpu().numpy())
        assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= 1.01e-10
    # A.D streams n(n+1)/2 + half the diagonal blocks per step instead of n^2 elements
    nb = -(-n // 128)
    diag = sum(min(128, n - 128 * K) ** 2 for K in range(nb))
    sym_step = 8 * 0.5 * (n * n + diag)
    steps = i_s["iters"]   # one A.D pass per block step (the stop test ends the step)
    assert abs(i_s["bytes_A"] - (steps * sym_step + (1 + 1 + i_s["restarts"]) * 8 * n * n)) <= 1.0


def test_pass_choice_is_part_of_the_captured_graph(gpu_ctx):
    """Solves of the same system with and without CCG_SYM_AD in one context each replay
    their own graphs: each gives the result of a fresh context with the same flags."""
    A, b, X0 = ci.system(1300, 4, 1e3, seed=2701)
    runs = [gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=f) for f in (CCG_SYM_AD, 0, CCG_SYM_AD, 0)]
    for f, (X, info) in zip((CCG_SYM_AD, 0), runs[:2]):
        fresh = Context(0)
        try:
            Xf, i_f = fresh.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=f)
        finally:
            fresh.close()
        assert info["iters"] == i_f["iters"] and torch.equal(X, Xf)
    assert torch.equal(runs[0][0], runs[2][0]) and torch.equal(runs[1][0], runs[3][0])
    assert not torch.equal(runs[0][0], runs[1][0])


def test_symmetric_profile_reports_triangle_bytes(gpu_ctx):
    n, p = 1500, 8
    A, b, X0 = ci.system(n, p, 1e3, seed=2401)
    gpu_ctx.kernel_time(reset=True)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=CCG_PROFILE | CCG_SYM_AD)
    ms, cnt, nbytes = gpu_ctx.kernel_time(reset=True, with_bytes=True)
    assert info["status"] == 0 and cnt == info["iters"] and ms > 0.0
    assert abs(nbytes / cnt - (8 * 0.5 * n * (n + 1) + 2 * 8 * n * p)) <= 1e-6 * nbytes / cnt
    gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=CCG_PROFILE)
    ms, cnt, nbytes = gpu_ctx.kernel_time(reset=True, with_bytes=True)
    assert abs(nbytes / cnt - (8.0 * n * n + 2 * 8 * n * p)) <= 1e-6 * nbytes / cnt


def test_strip_list_follows_n_in_one_workspace(gpu_ctx):
    """n = 1500 and n = 1100 share the padded size 1536 (one workspace), but not the
    block count: the second solve must rebuild the strip list and give the result of a
    fresh context."""
    A1, b1, X1 = ci.system(1500, 4, 1e2, seed=2501)
    A2, b2, X2 = ci.system(1100, 4, 1e2, seed=2502)
    gpu_ctx.solve(_t(A1), _t(b1), _t(X1), 1e-10, 20000, flags=CCG_SYM_AD)
    Xa, ia = gpu_ctx.solve(_t(A2), _t(b2), _t(X2), 1e-10, 20000, flags=CCG_SYM_AD)
    fresh = Context(0)
    try:
        Xb, ib = fresh.solve(_t(A2), _t(b2), _t(X2), 1e-10, 20000, flags=CCG_SYM_AD)
    finally:
        fresh.close()
    assert ia["status"] == 0 and ia["iters"] == ib["iters"] and torch.equal(Xa, Xb)


def test_symmetric_pass_is_deterministic(gpu_ctx):
    A, b, X0 = ci.system(2100, 8, 1e3, seed=2601)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=CCG_SYM_AD)
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, flags=CCG_SYM_AD)
    assert i1["iters"] == i2["iters"] and torch.equal(X1, X2)
