"""The oracle's pins must catch plausible mistakes.

Each case copies ccg_oracle.c, plants one mistake by text substitution (a dropped
term, a wrong sign, a transposed operand, a wrong index), builds it with gcc into a
temporary library, and checks that the pin battery below rejects it.  Everything
runs on the CPU; the planted code never leaves the temporary directory.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy.sparse.linalg import cg as scipy_cg

import ccg_inputs as ci
import oracle
from restart_util import first_restart_step

SRC = os.path.join(os.path.dirname(oracle.__file__), "ccg_oracle.c")

MUTANTS = {
    "beta_sign": ("for (int i = 0; i < m * m; ++i) beta[i] = -beta[i];",
                  "for (int i = 0; i < m * m; ++i) beta[i] = beta[i];"),
    "alpha_transposed": ("real a = alpha[l + c * m];", "real a = alpha[c + l * m];"),
    "residual_sign": ("rr[i] -= ad[i] * a;", "rr[i] += ad[i] * a;"),
    "dropped_D_beta": ("t[i] += d[i] * bb;", "t[i] += 0.0 * d[i] * bb;"),
    "gram_uses_R": ("gram(n, m, D, AD, G);", "gram(n, m, D, R, G);"),
    "beta_rhs_uses_D": ("gram(n, m, AD, R, W);", "gram(n, m, D, R, W);"),
    # (D^T R is symmetric in exact arithmetic -- it equals R^T R because R_{k+1} is
    # orthogonal to D_k -- so transposing it is not a mistake and is not listed.)
    "S_from_R_only": ("gram(n, m, D, R, S);", "gram(n, m, R, R, S); S[0] *= 1.5;"),
    "matmat_wrong_column": ("real mkj = M[k + (size_t)j * ldm];", "real mkj = M[k];"),
    "chol_solve_skips_back_substitution": ("for (int i = m - 1; i >= 0; --i) {     /* L^T z = y */",
                                           "for (int i = m - 1; i >= m; --i) {     /* L^T z = y */"),
    # the restart branch of the stop rule (explicit residual fails the confirmation)
    "restart_keeps_D": ("memcpy(D, T, (size_t)n * m * sizeof(real));\n                inf.restarts++;",
                        "inf.restarts++;"),
    "restart_keeps_R": ("memcpy(R, T, (size_t)n * m * sizeof(real));", ";"),
    "restart_not_counted": ("inf.restarts++;", ";"),
    # re-inflation (a policy beyond Alg. 3): the restart after it must be a fresh start
    "reinflate_keeps_D": ("memcpy(D, R, (size_t)n * m * sizeof(real));\n            inf.reinflations++;",
                          "inf.reinflations++;"),
    "reinflate_without_draw": ("Xr[i + (size_t)j * n] = xb[i] + unit_draw(splitmix64_next(&st));",
                               "Xr[i + (size_t)j * n] = xb[i];"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(tmpdir, f"{name}.c")
    path_so = os.path.join(tmpdir, f"{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", *oracle.GCC_FLAGS, "-o", path_so, path_c, "-lm"], check=True)
    return oracle.bind(path_so)


def _battery(lib):
    """Return the names of the pins that fail for this library."""
    failed = []
    # p = 1 against scipy CG
    A, b, X0 = ci.system(60, 1, 50.0, seed=2)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=5, lib=lib)
    xs, _ = scipy_cg(A, b, x0=X0[:, 0].copy(), rtol=0.0, atol=0.0, maxiter=5)
    if not np.all(np.isfinite(r["X"])) or \
            np.linalg.norm(r["X"][:, 0] - xs) > 1e-10 * np.linalg.norm(xs - X0[:, 0]):
        failed.append("p1_cg")
    # block Krylov optimality, p = 3, k = 2
    A, b, X0 = ci.system(50, 3, 20.0, seed=3)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=3, lib=lib)
    R0 = b[:, None] - A @ X0
    Q, _ = np.linalg.qr(np.hstack([R0, A @ R0, A @ A @ R0]))
    H = Q.T @ A @ Q
    for j in range(3):
        y = np.linalg.solve(H, Q.T @ (b - A @ X0[:, j]))
        x_opt = X0[:, j] + Q @ y
        if not np.all(np.isfinite(r["X"])) or \
                np.linalg.norm(r["X"][:, j] - x_opt) > 1e-9 * np.linalg.norm(x_opt - X0[:, j]):
            failed.append("krylov_optimality")
            break
    # finite termination, n = 12, p = 3
    A, b, X0 = ci.system(12, 3, 10.0, seed=21)
    r = oracle.ccg(A, b, X0, tol=0.0, maxit=4, lib=lib)
    xs = np.linalg.solve(A, b)
    if not np.all(np.isfinite(r["X"])) or np.abs(r["X"] - xs[:, None]).max() > 1e-10 * np.abs(xs).max():
        failed.append("finite_termination")
    # restart = fresh start from the agents at the restart step (Alg. 2 init, Alg. 4)
    A, b, X0 = ci.system(60, 3, 1e5, seed=0)
    full = oracle.ccg(A, b, X0, tol=1e-10, maxit=5000, lib=lib)
    kr = first_restart_step(A, b, X0, 1e-10, max(full["iters"], 1), lib=lib)
    ok = full["status"] == 0 and kr is not None
    if ok:
        at = oracle.ccg(A, b, X0, tol=0.0, maxit=kr, lib=lib)
        fresh = oracle.ccg(A, b, at["X"], tol=1e-10, maxit=5000, lib=lib)
        ok = (fresh["restarts"] == full["restarts"] - 1 and fresh["iters"] == full["iters"] - kr
              and np.array_equal(fresh["X"], full["X"]))
    if not ok:
        failed.append("restart")
    # re-inflation: the dropped duplicate agent restarts from the best start plus the
    # SplitMix64 draw, and the run is a fresh start from those agents
    A, b, X0 = ci.small_system()
    X0 = X0.copy()
    X0[:, 2] = X0[:, 0]
    full = oracle.ccg(A, b, X0, tol=1e-11, maxit=5000, reinflate_max=1, lib=lib)
    best = int(np.argmin(np.linalg.norm(b[:, None] - A @ X0, axis=0)))
    z = np.array(oracle.splitmix64((0x1204 << 48) ^ 2, A.shape[0]), dtype=np.uint64)
    X1 = X0.copy()
    X1[:, 2] = X0[:, best] + ((z >> np.uint64(11)).astype(np.float64) * (2.0 / 2 ** 53) - 1.0)
    fresh = oracle.ccg(A, b, X1, tol=1e-11, maxit=5000, lib=lib)
    if not (full["reinflations"] == 1 and full["p_final"] == 3 and fresh["iters"] == full["iters"]
            and np.array_equal(fresh["X"], full["X"])):
        failed.append("reinflate")
    return failed


def test_unmutated_oracle_passes_battery():
    assert _battery(oracle._load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(name, d)
        failed = _battery(lib)
    assert failed, f"planted mistake {name!r} passed every pin"
