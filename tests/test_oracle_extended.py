"""Pins of the oracle's extended-precision build (the same source, every internal
value in x86 80-bit extended precision), which the GPU parity tests use to measure
how far an FP64 trajectory has drifted from the method's own trajectory.

It must compute the same algorithm (p = 1 is textbook CG, the block-Krylov
optimality of each agent, the exact-rational golden run) and must really carry more
bits than the FP64 build: against the exact-rational run its error is far smaller.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.sparse.linalg import cg as scipy_cg

import ccg_inputs as ci
import oracle
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ld():
    return oracle.extended()


@pytest.mark.parametrize("k", [1, 3, 8, 21])
def test_p1_iterates_match_scipy_cg(ld, k):
    A, b, X0 = ci.system(120, 1, 100.0, seed=11)
    res = oracle.ccg(A, b, X0, tol=0.0, maxit=k, lib=ld)
    x_sp, _ = scipy_cg(A, b, x0=X0[:, 0].copy(), rtol=0.0, atol=0.0, maxiter=k)
    assert res["iters"] == k
    assert np.linalg.norm(res["X"][:, 0] - x_sp) <= 1e-10 * np.linalg.norm(x_sp - X0[:, 0])


@pytest.mark.parametrize("k", [1, 3])
def test_each_agent_optimal_on_block_krylov_space(ld, k):
    """X_{k+1} e_j minimises 1/2 x^T A x - b^T x on X0 e_j + span[R0, ..., A^k R0]."""
    A, b, X0 = ci.system(70, 3, 20.0, seed=3)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=k + 1, lib=ld)
    R0 = b[:, None] - A @ X0
    blocks = [R0]
    for _ in range(k):
        blocks.append(A @ blocks[-1])
    Q, _ = np.linalg.qr(np.hstack(blocks))
    H = Q.T @ A @ Q
    for j in range(3):
        y = np.linalg.solve(H, Q.T @ (b - A @ X0[:, j]))
        x_opt = X0[:, j] + Q @ y
        assert np.linalg.norm(r["X"][:, j] - x_opt) <= 1e-9 * np.linalg.norm(x_opt - X0[:, j])


def test_converges_to_direct_solve(ld):
    A, b, X0 = ci.small_system()
    res = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000, lib=ld)
    assert res["status"] == 0
    xs = np.linalg.solve(A, b)
    T = b[:, None] - A @ res["X"]
    rel = np.linalg.norm(T, axis=0) / np.linalg.norm(b)
    assert rel.min() <= 1.01e-10
    j = res["best_agent"]
    assert np.linalg.norm(res["X"][:, j] - xs) <= 1e3 * 1e-10 * np.linalg.norm(xs)


def _golden():
    with open(os.path.join(GOLDEN, "exact_ccg_n6_p2.json")) as f:
        g = json.load(f)
    fr = lambda s: float(Fraction(s))
    A = np.array(g["A"], dtype=np.float64)
    b = np.array(g["b"], dtype=np.float64)
    X0 = np.array(g["X0"], dtype=np.float64)
    ea = np.array([[[fr(v) for v in row] for row in a] for a in g["alphas"]])
    return A, b, X0, ea


def test_matches_exact_golden_and_carries_more_bits(ld):
    """The exact-rational run of the golden file: the extended build matches it
    to 1e-12, and its worst step-size error is at most 1/64 of the FP64 build's
    (11 more significand bits)."""
    A, b, X0, ea = _golden()
    steps = ea.shape[0] - 1        # the last step's beta is exactly zero
    r64 = oracle.ccg(A, b, X0, tol=0.0, maxit=steps, trace_k=steps)
    rld = oracle.ccg(A, b, X0, tol=0.0, maxit=steps, trace_k=steps, lib=ld)
    e64 = np.abs(r64["alphas"] - ea[:steps]).max() / np.abs(ea).max()
    eld = np.abs(rld["alphas"] - ea[:steps]).max() / np.abs(ea).max()
    assert eld <= 1e-12
    assert e64 > 0.0 and eld <= e64 / 64


def test_more_bits_on_a_larger_system(ld):
    """n = 8, four steps against the exact-rational routine: the extended build is
    closer at every step, and both agree with it."""
    A, b, X0 = ci.integer_system(8, 2, 3)
    run = exact.ccg(A, b, X0, steps=4)
    ea = np.array([[[float(v) for v in row] for row in a] for a in run["alphas"]])
    args = (np.array(A, float), np.array(b, float), np.array(X0, float))
    r64 = oracle.ccg(*args, tol=0.0, maxit=4, trace_k=4)
    rld = oracle.ccg(*args, tol=0.0, maxit=4, trace_k=4, lib=ld)
    e64 = np.abs(r64["alphas"] - ea).max()
    eld = np.abs(rld["alphas"] - ea).max()
    assert eld <= 1e-8 * np.abs(ea).max()
    assert eld < e64
