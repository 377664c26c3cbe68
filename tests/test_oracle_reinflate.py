"""Pins of the oracle's re-inflation policy (beyond Alg. 3): when the rank step would
drop some agents, each dropped agent restarts from the best active iterate plus a
SplitMix64 draw in [-1, 1) per entry, and the whole block restarts as Alg. 2 starts.

* The generator gives SplitMix64's published first outputs from state 0.
* A run that re-inflates equals, bit for bit, a plain run started from the
  re-inflated agents (the restart is Alg. 2's start, nothing more).
* Re-inflation keeps all p agents and still reaches the explicit-residual target.
"""
import numpy as np

import ccg_inputs as ci
import oracle


def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 seeded with 0 (Steele, Lea and Flood, OOPSLA 2014;
    # the reference sequence of that generator)
    assert oracle.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _draw(e, j, n):
    state = (0x1204 << 48) ^ (e << 32) ^ j
    z = np.array(oracle.splitmix64(state, n), dtype=np.uint64)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 2 ** 53) - 1.0


def _duplicate_start():
    A, b, X0 = ci.small_system()
    X0 = X0.copy()
    X0[:, 2] = X0[:, 0]
    return A, b, X0


def test_reinflated_run_is_a_fresh_start_from_the_new_agents():
    A, b, X0 = _duplicate_start()
    tol = 1e-11
    full = oracle.ccg(A, b, X0, tol=tol, maxit=5000, reinflate_max=1)
    assert full["status"] == 0 and full["reinflations"] == 1 and full["deflations"] == 0
    assert full["p_final"] == 3
    # at step 0 the rank step keeps agents 0 and 1 (agent 2 duplicates agent 0); the
    # best of the three starting residuals gives the base of agent 2's new start
    best = int(np.argmin(np.linalg.norm(b[:, None] - A @ X0, axis=0)))
    X1 = X0.copy()
    X1[:, 2] = X0[:, best] + _draw(0, 2, A.shape[0])
    fresh = oracle.ccg(A, b, X1, tol=tol, maxit=5000)
    assert fresh["iters"] == full["iters"] and fresh["reinflations"] == 0
    assert np.array_equal(fresh["X"], full["X"])


def test_without_reinflation_the_agent_is_dropped():
    A, b, X0 = _duplicate_start()
    plain = oracle.ccg(A, b, X0, tol=1e-11, maxit=5000)
    assert plain["deflations"] == 1 and plain["p_final"] == 2 and plain["reinflations"] == 0


def test_reinflation_budget_and_convergence():
    """Rank drops of floating point near the end of a run (p not dividing n): with a
    budget of 3 the run re-inflates at most 3 times, then drops agents as Alg. 3 does,
    and still meets tol; without a budget it drops them at once."""
    for n, p, seed in [(13, 3, 21), (100, 8, 3)]:
        A, b, X0 = ci.system(n, p, 10.0, seed=seed)
        tol = 1e-10
        plain = oracle.ccg(A, b, X0, tol=tol, maxit=5000)
        re = oracle.ccg(A, b, X0, tol=tol, maxit=5000, reinflate_max=3)
        assert plain["deflations"] >= 1 and plain["reinflations"] == 0
        assert 1 <= re["reinflations"] <= 3
        for r in (plain, re):
            T = b[:, None] - A @ r["X"]
            assert r["status"] == 0
            assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= tol
