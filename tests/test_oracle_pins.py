"""Pins for the oracle: facts the paper and the mathematics fix, none of them a
re-typing of the oracle's own formulas.

* p = 1 is textbook CG (Sec. 3.2: cCG generalises CG) -> scipy's CG iterates.
* The converged answer is x* = A^{-1} b (Sec. 2) -> LAPACK solve, with the bound
  ||x - x*|| / ||x*|| <= cond(A) * ||b - A x|| / ||b||.
* Theorem 2 (properties of cCG): residual blocks mutually orthogonal, direction
  blocks mutually A-orthogonal, and each agent optimal on X0 e_j + block Krylov
  space -> brute-force Galerkin solve on that space.
* Theorem 3 (genericity): when p divides n the run ends after n/p steps; when it
  does not, D loses rank at floor(n/p) and the rank step (Alg. 3) takes over.
* Exact arithmetic: the FP64 oracle agrees step by step with the exact-rational
  run, which itself ends with R == 0 exactly and X == A^{-1} b exactly.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
from scipy.sparse.linalg import cg as scipy_cg

import ccg_inputs as ci
import oracle
from oracle import exact
from restart_util import first_restart_step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sys(n, p, kappa, seed=11):
    return ci.system(n, p, kappa, seed=seed)


# ------------------------------------------------------------------ p = 1 is CG

@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 21])
def test_p1_iterates_match_scipy_cg(k):
    A, b, X0 = _sys(120, 1, 100.0)
    res = oracle.ccg(A, b, X0, tol=0.0, maxit=k)
    x_sp, _ = scipy_cg(A, b, x0=X0[:, 0].copy(), rtol=0.0, atol=0.0, maxiter=k)
    x_or = res["X"][:, 0]
    assert res["iters"] == k
    scale = np.linalg.norm(x_sp - X0[:, 0])
    assert np.linalg.norm(x_or - x_sp) <= 1e-10 * scale


def test_p1_converges_like_cg():
    A, b, X0 = _sys(200, 1, 1e3)
    res = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000)
    assert res["status"] == 0
    x_sp, info = scipy_cg(A, b, x0=X0[:, 0].copy(), rtol=1e-10, atol=0.0, maxiter=5000)
    assert info == 0
    # same Krylov method: iteration counts within a few steps of each other
    it_sp = []
    scipy_cg(A, b, x0=X0[:, 0].copy(), rtol=1e-10, atol=0.0, maxiter=5000,
             callback=lambda xk: it_sp.append(1))
    assert abs(res["iters"] - len(it_sp)) <= max(5, len(it_sp) // 20)


# ------------------------------------------------------- converged answer is x*

@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_small_system_converges_to_direct_solve(p):
    A, b, X0 = ci.small_system(p=p)
    kappa = 1e3
    res = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000)
    assert res["status"] == 0, res["status_name"]
    xs = scipy.linalg.solve(A, b, assume_a="pos")
    X = res["X"]
    T = b[:, None] - A @ X          # numpy residual, independent of the oracle's
    rel = np.linalg.norm(T, axis=0) / np.linalg.norm(b)
    assert rel.min() <= 1e-10
    assert res["best_agent"] == int(np.argmin(rel))
    assert abs(res["rel_res"] - rel.min()) <= 1e-3 * rel.min()
    err = np.linalg.norm(X - xs[:, None], axis=0) / np.linalg.norm(xs)
    assert np.all(err <= 1.01 * kappa * rel + 1e-14)
    assert err[res["best_agent"]] <= kappa * 1e-10


def test_cooperation_needs_fewer_steps_than_cg():
    """More agents -> fewer block steps (Sec. 5: about 1.6x fewer at p = 3)."""
    A, b, X0 = ci.small_system(p=3)
    r1 = oracle.ccg(A, b, X0[:, :1], tol=1e-10, maxit=5000)
    r3 = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000)
    assert r3["iters"] < r1["iters"]


# ---------------------------------------------- Theorem 2 (properties of cCG)

def _trajectory(A, b, X0, kmax):
    Rs, Ds, Xs = [], [], []
    for k in range(kmax + 1):
        r = oracle.ccg(A, b, X0, tol=0.0, maxit=k, want_rd=True)
        Rs.append(r["R"])
        Ds.append(r["D"])
        Xs.append(r["X"])
    return Xs, Rs, Ds


def test_block_orthogonality_and_conjugacy():
    A, b, X0 = _sys(60, 3, 10.0, seed=5)
    Xs, Rs, Ds = _trajectory(A, b, X0, 6)
    for i in range(7):
        for j in range(7):
            if i == j:
                continue
            ri = Rs[i] / np.linalg.norm(Rs[i], axis=0)
            rj = Rs[j] / np.linalg.norm(Rs[j], axis=0)
            assert np.abs(ri.T @ rj).max() <= 1e-10, (i, j)
            di = Ds[i] / np.sqrt(np.einsum("ij,ij->j", Ds[i], A @ Ds[i]))
            dj = Ds[j] / np.sqrt(np.einsum("ij,ij->j", Ds[j], A @ Ds[j]))
            assert np.abs(di.T @ A @ dj).max() <= 1e-10, (i, j)
            if j < i:   # residual orthogonal to earlier directions
                dn = Ds[j] / np.linalg.norm(Ds[j], axis=0)
                assert np.abs(ri.T @ dn).max() <= 1e-10


def test_recurrence_residual_equals_explicit_residual_early():
    A, b, X0 = _sys(80, 4, 50.0, seed=9)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=5, want_rd=True)
    T = b[:, None] - A @ r["X"]
    assert np.abs(T - r["R"]).max() <= 1e-10 * np.abs(T).max() * 1e3


@pytest.mark.parametrize("k", [0, 1, 3, 6])
def test_each_agent_optimal_on_block_krylov_space(k):
    """X_{k+1} e_j minimises f on X0 e_j + span[R0, A R0, ..., A^k R0]."""
    A, b, X0 = _sys(70, 3, 20.0, seed=3)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=k + 1)
    R0 = b[:, None] - A @ X0
    blocks = [R0]
    for _ in range(k):
        blocks.append(A @ blocks[-1])
    Q, _ = np.linalg.qr(np.hstack(blocks))
    H = Q.T @ A @ Q
    for j in range(3):
        y = np.linalg.solve(H, Q.T @ (b - A @ X0[:, j]))
        x_opt = X0[:, j] + Q @ y
        scale = np.linalg.norm(x_opt - X0[:, j])
        assert np.linalg.norm(r["X"][:, j] - x_opt) <= 1e-9 * scale, (k, j)


# ------------------------------------------ Theorem 3 (genericity), Alg. 3 (mcCG)

def test_finite_termination_when_p_divides_n():
    A, b, X0 = _sys(12, 3, 10.0, seed=21)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=4, want_rd=True)
    assert np.linalg.norm(r["R"]) <= 1e-12 * np.linalg.norm(b)
    xs = np.linalg.solve(A, b)
    assert np.abs(r["X"] - xs[:, None]).max() <= 1e-12 * np.abs(xs).max()


def test_rank_drop_when_p_does_not_divide_n():
    A, b, X0 = _sys(13, 3, 10.0, seed=21)
    r = oracle.ccg(A, b, X0, tol=1e-12, maxit=50)
    assert r["status"] == 0
    assert r["deflations"] >= 1 and r["p_final"] < 3
    # after the rank step at floor(13/3) = 4 steps, CG needs at most p-1 more
    assert r["iters"] <= 4 + 2
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(r["X"][:, r["best_agent"]] - xs) <= 1e-10 * np.linalg.norm(xs)


def test_duplicate_start_columns_deflate_at_step_zero():
    A, b, X0 = ci.small_system(p=3)
    X0 = X0.copy()
    X0[:, 2] = X0[:, 0]
    r = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000)
    assert r["status"] == 0
    assert r["deflations"] >= 1 and r["p_final"] == 2
    T = b[:, None] - A @ r["X"]
    assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= 1e-10


# ------------------------------- stop rule of Alg. 4: confirmation and restart

RESTART_CASES = [(60, 3, 1e5, 0), (60, 2, 1e6, 3), (300, 3, 1e6, 7)]


@pytest.mark.parametrize("n,p,kappa,seed", RESTART_CASES)
def test_restart_continues_as_a_fresh_start(n, p, kappa, seed):
    """When the recurrence residual passes the stop test but the explicit residual
    B - A X does not, the run restarts.  Alg. 2's first lines define what a start
    from X is (R = B - A X, D = R), so the rest of the run must equal, bit for bit,
    a fresh run started from the agents at the restart step, and the count of
    restarts must be that fresh run's count plus one."""
    A, b, X0 = ci.system(n, p, kappa, seed=seed)
    tol = 1e-10
    full = oracle.ccg(A, b, X0, tol=tol, maxit=50000)
    assert full["status"] == 0 and full["restarts"] >= 1 and full["deflations"] == 0
    kr = first_restart_step(A, b, X0, tol, full["iters"])
    assert kr is not None and 0 < kr < full["iters"]
    at = oracle.ccg(A, b, X0, tol=0.0, maxit=kr, want_rd=True)
    nb = np.linalg.norm(b)
    # at step kr the recurrence residual passes the test (numpy norms) ...
    assert (np.linalg.norm(at["R"], axis=0) / nb).min() <= tol
    # ... while the explicit residual, formed by numpy, fails it
    T = b[:, None] - A @ at["X"]
    assert (np.linalg.norm(T, axis=0) / nb).min() > tol
    fresh = oracle.ccg(A, b, at["X"], tol=tol, maxit=50000)
    assert fresh["status"] == 0
    assert fresh["restarts"] == full["restarts"] - 1
    assert fresh["iters"] == full["iters"] - kr
    assert np.array_equal(fresh["X"], full["X"])


# ------------------------------------------------------------- error handling

def test_errors():
    A, b, X0 = _sys(30, 2, 10.0)
    bn = b.copy()
    bn[3] = np.nan
    assert oracle.ccg(A, bn, X0, 1e-8, 100)["status"] == -2
    assert oracle.ccg(-np.eye(30), b, X0, 1e-8, 100)["status"] == -3
    assert oracle.ccg(A, b, X0, -1.0, 100)["status"] == -1
    assert oracle.ccg(A, np.zeros(30), X0, 1e-8, 100)["status"] == -1
    r = oracle.ccg(A, b, X0, 1e-14, 1)
    assert r["status"] == 1 and r["iters"] == 1


# -------------------------------------------------------------- exact arithmetic

def _exact_system(n, p, seed):
    return ci.integer_system(n, p, seed)


def _fmat(M):
    return [[Fraction(v) for v in row] for row in M]


@pytest.mark.parametrize("n,p,seed", [(6, 2, 7), (6, 3, 1), (8, 4, 2), (9, 3, 4)])
def test_exact_run_terminates_with_zero_residual(n, p, seed):
    A, b, X0 = _exact_system(n, p, seed)
    run = exact.ccg(A, b, X0, steps=n // p)
    R = run["Rs"][-1]
    assert all(v == 0 for row in R for v in row)
    xs = exact.solve(_fmat(A), [[Fraction(v)] for v in b])
    X = run["Xs"][-1]
    assert all(X[i][j] == xs[i][0] for i in range(n) for j in range(p))
    # Theorem 2: exact block orthogonality / A-conjugacy
    Af = _fmat(A)
    Rs, Ds = run["Rs"], run["Ds"]
    for i in range(len(Rs) - 1):
        for j in range(i):
            assert all(v == 0 for row in exact.matmul(exact.transpose(Rs[i]), Rs[j]) for v in row)
            ADj = exact.matmul(Af, Ds[j])
            assert all(v == 0 for row in exact.matmul(exact.transpose(Ds[i]), ADj) for v in row)


def test_exact_rank_drop_when_p_does_not_divide_n():
    A, b, X0 = _exact_system(7, 3, 5)
    run = exact.ccg(A, b, X0, steps=4)
    assert run["stopped_rank"] is not None and run["stopped_rank"] < 3
    assert len(run["alphas"]) == 7 // 3


def test_fp64_oracle_matches_exact_golden():
    with open(os.path.join(GOLDEN, "exact_ccg_n6_p2.json")) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.float64)
    b = np.array(g["b"], dtype=np.float64)
    X0 = np.array(g["X0"], dtype=np.float64)
    steps = len(g["alphas"])
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=steps, trace_k=steps)

    def fr(s):
        return float(Fraction(s))

    ea = np.array([[[fr(v) for v in row] for row in a] for a in g["alphas"]])
    eb = np.array([[[fr(v) for v in row] for row in bt] for bt in g["betas"]])
    # the last beta is exactly zero (R vanishes), so scale by the whole run
    assert np.abs(r["alphas"] - ea).max() <= 1e-9 * np.abs(ea).max()
    assert np.abs(r["betas"] - eb).max() <= 1e-9 * np.abs(eb).max()
    xe = np.array([[fr(v) for v in row] for row in g["X_final"]])
    assert np.abs(r["X"] - xe).max() <= 1e-9 * np.abs(xe).max()
    # golden file is itself consistent with the exact routine
    run = exact.ccg(g["A"], g["b"], g["X0"], steps=steps)
    assert [[f"{v.numerator}/{v.denominator}" for v in row] for row in run["alphas"][0]] == \
        g["alphas"][0]


def test_fp64_oracle_matches_exact_every_step():
    A, b, X0 = _exact_system(8, 2, 3)
    run = exact.ccg(A, b, X0, steps=4)
    r = oracle.ccg(np.array(A, float), np.array(b, float), np.array(X0, float),
                   tol=0.0, maxit=4, trace_k=4)
    ea = np.array([[[float(v) for v in row] for row in a] for a in run["alphas"]])
    eb = np.array([[[float(v) for v in row] for row in bt] for bt in run["betas"]])
    for k in range(4):
        assert np.abs(r["alphas"][k] - ea[k]).max() <= 1e-8 * np.abs(ea).max(), k
        assert np.abs(r["betas"][k] - eb[k]).max() <= 1e-8 * np.abs(eb).max(), k
