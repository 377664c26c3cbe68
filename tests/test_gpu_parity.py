"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP64 mode):
  * per block step, alpha_k and beta_k agree to 1e-10 relative to the step's largest
    entry, and X, R, D to 1e-10 relative to each block's norm (the two sides sum in
    different orders; observed gaps are ~1e-14 for the first steps);
  * a full solve: after about 50 steps block CG in floating point decorrelates the
    residual directions of any two summation orders (the oracle against numpy's
    BLAS order shows the same), while the iterates converge together.  So the GPU
    run is compared with the oracle run for the SAME number of steps.  Taken to a
    relative residual of 1e-11, every agent column agrees to 1e-10 relative (the
    bound the solver is held to; oracle vs numpy gaps measure <= 3e-12 there).
    Stopped at 1e-10, both iterates still carry up to cond(A) * 1e-10 of error in
    the slow eigen-directions, so the gap is held to the arithmetic bound
    2 * cond(A) * tol (measured: 1.4e-10 at n=256).  In both cases the natural
    stopping steps agree within 5 % and the explicit FP64 residual is <= tol.
"""
import numpy as np
import pytest
import torch

import ccg_inputs as ci
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


STEP_CASES = [
    (256, 3, 1e3, 10),    # the n=256, p=3 workload; one row tile
    (1000, 5, 1e3, 8),    # ragged tail tile, p padded to 8
    (777, 2, 1e2, 6),     # odd n
    (2085, 8, 1e4, 5),    # several tiles and splits, ragged
    (300, 1, 1e3, 10),    # p = 1 (CG)
    (640, 16, 1e2, 4),    # largest p
    (129, 4, 10.0, 6),
]


@pytest.mark.parametrize("n,p,kappa,k", STEP_CASES)
def test_debug_steps_match_oracle(gpu_ctx, n, p, kappa, k):
    print(f"case debug_step n={n} p={p} kappa={kappa} k={k}", flush=True)
    A, b, X0 = ci.system(n, p, kappa, seed=101)
    orc = oracle.ccg(A, b, X0, tol=0.0, maxit=k, trace_k=k, want_rd=True)
    g = gpu_ctx.debug_step(_t(A), _t(b), _t(X0), k)
    for s in range(k):
        sa = np.abs(orc["alphas"][s]).max()
        sb = np.abs(orc["betas"][s]).max()
        assert np.abs(g["alphas"][s] - orc["alphas"][s]).max() <= 1e-10 * sa, ("alpha", s)
        assert np.abs(g["betas"][s] - orc["betas"][s]).max() <= 1e-10 * sb, ("beta", s)
    assert _rel(g["X"].numpy(), orc["X"]) <= 1e-10
    assert _rel(g["R"].numpy(), orc["R"]) <= 1e-10
    assert _rel(g["D"].numpy(), orc["D"]) <= 1e-10


SOLVE_CASES = [
    (256, 3, 1e3),
    (1000, 4, 1e3),
    (513, 2, 1e2),
    (300, 1, 1e2),
    (700, 8, 1e3),
]


def _check_against_oracle(A, b, X0, X, info, tol, orc_natural=None, gap=1e-10):
    """Same-step comparison (see module docstring) plus explicit-residual checks."""
    Xg = X.cpu().numpy()
    p = Xg.shape[1]
    if orc_natural is not None:
        ko = orc_natural["iters"]
        assert abs(info["iters"] - ko) <= max(3, 0.05 * ko), (info["iters"], ko)
    if info["restarts"] == 0:
        same = oracle.ccg(A, b, X0, tol=0.0, maxit=info["iters"])
        assert same["p_final"] == info["p_final"]
        for j in range(p):
            assert _rel(Xg[:, j], same["X"][:, j]) <= gap, j
    T = b[:, None] - A @ Xg
    rel = np.linalg.norm(T, axis=0) / np.linalg.norm(b)
    if info["status"] == 0:
        assert rel.min() <= tol
    # b - A x near 1e-11 * ||b|| loses digits to cancellation: two summation orders
    # differ by ~1e-15 * ||b|| (absolute), so compare at that level.
    assert abs(info["rel_res"] - rel.min()) <= 1e-3 * rel.min() + 1e-14
    assert rel[info["best_agent"]] <= rel.min() * (1 + 1e-3) + 1e-14


@pytest.mark.parametrize("n,p,kappa", SOLVE_CASES)
def test_solve_matches_oracle(gpu_ctx, n, p, kappa):
    print(f"case solve n={n} p={p} kappa={kappa}", flush=True)
    if n == 256 and p == 3:
        A, b, X0 = ci.small_system()
    else:
        A, b, X0 = ci.system(n, p, kappa, seed=202)
    tol = 1e-11
    orc = oracle.ccg(A, b, X0, tol=tol, maxit=20000)
    assert orc["status"] == 0
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), tol, 20000)
    assert info["status"] == 0, info
    _check_against_oracle(A, b, X0, X, info, tol, orc)


@pytest.mark.parametrize("n,p,kappa", [(256, 3, 1e3), (700, 8, 1e3)])
def test_solve_at_benchmark_tolerance(gpu_ctx, n, p, kappa):
    print(f"case solve tol=1e-10 n={n} p={p} kappa={kappa}", flush=True)
    if n == 256 and p == 3:
        A, b, X0 = ci.small_system()
    else:
        A, b, X0 = ci.system(n, p, kappa, seed=202)
    tol = 1e-10
    orc = oracle.ccg(A, b, X0, tol=tol, maxit=20000)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), tol, 20000)
    assert info["status"] == 0, info
    _check_against_oracle(A, b, X0, X, info, tol, orc, gap=2 * kappa * tol)


def test_solve_is_deterministic(gpu_ctx):
    A, b, X0 = ci.system(1500, 4, 1e3, seed=5)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000)
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000)
    assert i1["iters"] == i2["iters"]
    assert torch.equal(X1, X2)


def test_graph_and_direct_launch_agree(gpu_ctx):
    from paper_1204_0069_amd import CCG_NO_GRAPH
    A, b, X0 = ci.system(900, 4, 1e3, seed=8)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000)
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000, flags=CCG_NO_GRAPH)
    assert i1["iters"] == i2["iters"]
    assert torch.equal(X1, X2)


def test_round_lengths_do_not_change_results(gpu_ctx):
    """FP64 rounds grow from graph_k up to 8 graph_k while the residual is far from tol;
    where they end must not change the steps: graph_k 1, 4 and 16 (rounds of 1..128
    steps, several graphs in one context) give the same result, and so does a solve
    after the other sizes' graphs were captured."""
    A, b, X0 = ci.system(2100, 6, 1e4, seed=9)
    runs = [gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, graph_k=k) for k in (16, 1, 4, 16)]
    for X, info in runs[1:]:
        assert info["status"] == 0 and info["iters"] == runs[0][1]["iters"]
        assert torch.equal(X, runs[0][0])
    assert runs[0][1]["iters"] > 128


def test_profiled_solves_agree_and_count_launches(gpu_ctx):
    """Timing the A.D launches (every round, or every 4th round with the rest from the
    graph) changes how steps are launched, not what they compute."""
    from paper_1204_0069_amd import CCG_PROFILE, CCG_PROFILE_SAMPLED
    A, b, X0 = ci.system(700, 3, 1e3, seed=9)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000)
    gpu_ctx.kernel_time(reset=True)
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000, flags=CCG_PROFILE)
    ms_all, n_all = gpu_ctx.kernel_time(reset=True)
    X3, i3 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 5000, flags=CCG_PROFILE_SAMPLED)
    ms_s, n_s = gpu_ctx.kernel_time(reset=True)
    assert i1["iters"] == i2["iters"] == i3["iters"]
    assert torch.equal(X1, X2) and torch.equal(X1, X3)
    assert i1["iters"] > 64                            # several rounds of 16 steps
    assert n_all == i1["iters"] + 1 + i1["restarts"]   # every launch that streamed A
    assert 0 < n_s < n_all                             # the launches of every 4th round
    assert ms_all > 0.0 and ms_s > 0.0


# ----------------------------------------------------------------- edge cases

def test_duplicate_columns_deflate(gpu_ctx):
    A, b, X0 = ci.small_system()
    X0 = X0.copy()
    X0[:, 2] = X0[:, 0]
    orc = oracle.ccg(A, b, X0, tol=1e-11, maxit=5000)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-11, 5000)
    assert info["status"] == 0
    assert info["deflations"] >= 1 and info["p_final"] == orc["p_final"] == 2
    _check_against_oracle(A, b, X0, X, info, 1e-11, orc)


def test_rank_drop_p_not_dividing_n(gpu_ctx):
    A, b, X0 = ci.system(13, 3, 10.0, seed=21)
    orc = oracle.ccg(A, b, X0, tol=1e-12, maxit=50)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-12, 50)
    assert info["status"] == 0
    assert info["deflations"] == orc["deflations"] >= 1
    assert info["p_final"] == orc["p_final"]
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(X.cpu().numpy()[:, info["best_agent"]] - xs) <= 1e-9 * np.linalg.norm(xs)


def test_tiny_systems(gpu_ctx):
    for n, p in [(1, 1), (2, 2), (5, 5), (16, 16), (17, 3)]:
        A, b, X0 = ci.system(n, p, 10.0, seed=n)
        orc = oracle.ccg(A, b, X0, tol=1e-12, maxit=100)
        X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-12, 100)
        assert info["status"] == orc["status"] == 0, (n, p, info)
        xs = np.linalg.solve(A, b)
        assert np.linalg.norm(X.cpu().numpy()[:, info["best_agent"]] - xs) <= 1e-9 * np.linalg.norm(xs)


def test_start_at_solution_needs_no_steps(gpu_ctx):
    A, b, X0 = ci.system(200, 2, 10.0, seed=3)
    xs = np.linalg.solve(A, b)
    X0 = np.stack([xs, xs + 1.0], axis=1)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100)
    assert info["status"] == 0 and info["iters"] == 0 and info["best_agent"] == 0


def test_maxit_reports_not_converged(gpu_ctx):
    A, b, X0 = ci.system(400, 3, 1e3, seed=4)
    orc = oracle.ccg(A, b, X0, tol=1e-12, maxit=7)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-12, 7)
    assert info["status"] == 1 and info["iters"] == 7
    assert _rel(X.cpu().numpy(), orc["X"]) <= 1e-10
    assert abs(info["rel_res"] - orc["rel_res"]) <= 1e-6 * orc["rel_res"]


def test_errors_are_reported(gpu_ctx):
    from paper_1204_0069_amd import CcgError
    A, b, X0 = ci.system(64, 2, 10.0, seed=1)
    bn = b.copy()
    bn[5] = np.nan
    X, info = gpu_ctx.solve(_t(A), _t(bn), _t(X0), 1e-10, 100, raise_on_error=False)
    assert info["status"] == -2
    X, info = gpu_ctx.solve(_t(-np.eye(64)), _t(b), _t(X0), 1e-10, 100, raise_on_error=False)
    assert info["status"] == -3
    with pytest.raises(CcgError):
        gpu_ctx.solve(_t(A), _t(b), _t(X0), -1.0, 100)
    with pytest.raises(CcgError):
        gpu_ctx.solve(_t(A), _t(b), _t(np.zeros((64, 17))), 1e-10, 100)
    # the context still works afterwards
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 200)
    assert info["status"] == 0


# ------------------------------------------------- full size: n=8192, p=8, kappa=1e4

@pytest.fixture(scope="module")
def big_system():
    n, p = 8192, 8
    A = ci.spd_spectrum(n, 1e4, ci.item_seed("A", 1204, base=n), device=DEV)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", 1204, base=n)), device=DEV)
    X0 = torch.as_tensor(ci.normal_block(n, p, ci.item_seed("X0", 1204, base=n)), device=DEV)
    return A, b, X0


def test_full_size_first_steps_match_oracle(gpu_ctx, big_system):
    A, b, X0 = big_system
    print("case full-size debug_step n=8192 p=8 k=2", flush=True)
    k = 2
    g = gpu_ctx.debug_step(A, b, X0, k)
    An = A.cpu().numpy()
    orc = oracle.ccg(An, b.cpu().numpy(), X0.cpu().numpy(), tol=0.0, maxit=k, trace_k=k,
                     want_rd=True)
    for s in range(k):
        assert np.abs(g["alphas"][s] - orc["alphas"][s]).max() <= 1e-10 * np.abs(orc["alphas"][s]).max()
        assert np.abs(g["betas"][s] - orc["betas"][s]).max() <= 1e-10 * np.abs(orc["betas"][s]).max()
    assert _rel(g["X"].numpy(), orc["X"]) <= 1e-10
    assert _rel(g["R"].numpy(), orc["R"]) <= 1e-10


def test_full_size_solve_properties(gpu_ctx, big_system):
    """At n=8192 the oracle would take minutes per solve; check what holds at any size:
    explicit FP64 residual (torch/rocBLAS, not the library) <= tol for the reported best
    agent, and the error bound against the direct solution."""
    A, b, X0 = big_system
    print("case full-size solve n=8192 p=8 kappa=1e4", flush=True)
    tol = 1e-10
    X, info = gpu_ctx.solve(A, b, X0, tol, 20000)
    assert info["status"] == 0, info
    T = b[:, None] - A @ X
    rel = (torch.linalg.norm(T, dim=0) / torch.linalg.norm(b)).cpu().numpy()
    assert rel[info["best_agent"]] <= tol
    assert abs(rel.min() - info["rel_res"]) <= 1e-3 * info["rel_res"] + 1e-14
    xs = torch.linalg.solve(A, b)
    err = (torch.linalg.norm(X[:, info["best_agent"]] - xs) / torch.linalg.norm(xs)).item()
    assert err <= 1e4 * tol


def test_small_solve_after_larger_one_in_same_workspace(gpu_ctx):
    """Regression: rows n..n_pad of the workspace must not carry values from an
    earlier, larger solve that used the same padded size."""
    A1, b1, X1 = ci.system(500, 3, 1e2, seed=31)
    gpu_ctx.solve(_t(A1), _t(b1), _t(X1), 1e-10, 2000)
    A, b, X0 = ci.system(13, 3, 10.0, seed=21)
    orc = oracle.ccg(A, b, X0, tol=1e-12, maxit=50)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-12, 50)
    assert info["status"] == 0 and info["iters"] == orc["iters"]
    assert info["deflations"] == orc["deflations"]


def test_inputs_are_not_modified(gpu_ctx):
    """X0 (including a single column, whose transpose shares its storage), A and b
    are read only."""
    for p in (1, 3):
        A, b, X0 = ci.system(200, p, 1e2, seed=31)
        At, bt, Xt = _t(A), _t(b), _t(X0)
        A0, b0, X00 = At.clone(), bt.clone(), Xt.clone()
        X, info = gpu_ctx.solve(At, bt, Xt, 1e-10, 5000)
        assert info["status"] == 0 and info["iters"] > 0
        assert torch.equal(At, A0) and torch.equal(bt, b0) and torch.equal(Xt, X00)
        g = gpu_ctx.debug_step(At, bt, Xt, 2)
        assert torch.equal(Xt, X00)


@pytest.mark.parametrize("pad", [2, 3, 64])
@pytest.mark.parametrize("n,p,prec,flags", [(1100, 5, "fp64", 0), (1100, 5, "fp64", "sym"), (700, 4, "fp32", 0),
                                          (700, 4, "bf16x2", 0)])
def test_leading_dimension_larger_than_n(gpu_ctx, n, p, prec, flags, pad):
    """A passed as the n x n corner of a larger array (lda = n + pad): an even pad keeps
    its columns 16-byte aligned and is streamed in place, an odd pad makes the library
    copy it to an aligned buffer first.  Either way the result equals that of the
    contiguous matrix, bit for bit."""
    from paper_1204_0069_amd import CCG_SYM_AD
    fl = CCG_SYM_AD if flags == "sym" else 0
    print(f"case lda n={n} pad={pad} p={p} {prec} flags={flags}", flush=True)
    A, b, X0 = ci.system(n, p, 1e3, seed=3100 + n + pad)
    big = torch.zeros(n + pad, n + pad, dtype=torch.float64, device=DEV)
    big[:n, :n] = _t(A)
    view = big[:n, :n]
    assert view.stride(0) == n + pad
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000, prec=prec, flags=fl)
    X2, i2 = gpu_ctx.solve(view, _t(b), _t(X0), 1e-10, 20000, prec=prec, flags=fl)
    assert i1["status"] == 0 and i2["status"] == 0
    assert i1["iters"] == i2["iters"] and torch.equal(X1, X2)
    assert torch.equal(big[:n, :n], _t(A)) and not big[n:, :].any() and not big[:, n:].any()
