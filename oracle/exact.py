"""Exact-arithmetic cooperative CG on tiny systems (Python fractions).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Alg. 2 of the paper (cCG, Sec. 3.2) in rational arithmetic, in the sign
convention R = B - A X:

    G = D^T A D,  alpha = G^{-1} D^T R,  X += D alpha,  R -= A D alpha,
    beta = -G^{-1} (A D)^T R,  D = R + D beta.

With exact arithmetic, Theorem 3 of the paper (genericity) says the run ends with
R = 0 after n/p steps when p divides n, and Theorem 2 (properties of cCG) says the
residual blocks are mutually orthogonal and the direction blocks mutually
A-orthogonal.  The tests check those facts exactly (zero, not small), which pins
this implementation; the FP64 C oracle is then compared against it step by step.

Matrices are lists of rows of ``Fraction``.  Pure-Python loops: keep n <= ~12.
"""
from __future__ import annotations

from fractions import Fraction


def _zeros(r, c):
    return [[Fraction(0)] * c for _ in range(r)]


def matmul(P, Q):
    r, k, c = len(P), len(Q), len(Q[0])
    out = _zeros(r, c)
    for i in range(r):
        for j in range(c):
            s = Fraction(0)
            for t in range(k):
                s += P[i][t] * Q[t][j]
            out[i][j] = s
    return out


def transpose(P):
    return [list(col) for col in zip(*P)]


def solve(G, B):
    """Exact Gauss-Jordan solve of G Z = B (G square, nonsingular)."""
    m = len(G)
    q = len(B[0])
    M = [list(G[i]) + list(B[i]) for i in range(m)]
    for c in range(m):
        piv = next(r for r in range(c, m) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(m):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [row[m:m + q] for row in M]


def rank(P):
    """Exact rank by row reduction."""
    M = [list(r) for r in P]
    rows, cols = len(M), len(M[0])
    rk = 0
    for c in range(cols):
        piv = next((r for r in range(rk, rows) if M[r][c] != 0), None)
        if piv is None:
            continue
        M[rk], M[piv] = M[piv], M[rk]
        for r in range(rows):
            if r != rk and M[r][c] != 0:
                f = M[r][c] / M[rk][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[rk])]
        rk += 1
    return rk


def ccg(A, b, X0, steps: int):
    """Run ``steps`` exact cCG steps (stops early if D loses rank).

    Returns a dict with lists Xs, Rs, Ds (the blocks after 0..k steps), alphas,
    betas, and ``stopped_rank`` (the rank of D where the run stopped, or None).
    """
    A = [[Fraction(v) for v in row] for row in A]
    n = len(A)
    X = [[Fraction(v) for v in row] for row in X0]
    p = len(X[0])
    AX = matmul(A, X)
    R = [[Fraction(b[i]) - AX[i][j] for j in range(p)] for i in range(n)]
    D = [list(r) for r in R]
    out = {"Xs": [X], "Rs": [R], "Ds": [D], "alphas": [], "betas": [], "stopped_rank": None}
    for _ in range(steps):
        rk = rank(D)
        if rk < p:
            out["stopped_rank"] = rk
            break
        AD = matmul(A, D)
        Dt = transpose(D)
        G = matmul(Dt, AD)
        alpha = solve(G, matmul(Dt, R))
        Dal = matmul(D, alpha)
        ADal = matmul(AD, alpha)
        X = [[X[i][j] + Dal[i][j] for j in range(p)] for i in range(n)]
        R = [[R[i][j] - ADal[i][j] for j in range(p)] for i in range(n)]
        beta = solve(G, matmul(transpose(AD), R))
        beta = [[-v for v in row] for row in beta]
        Dbe = matmul(D, beta)
        D = [[R[i][j] + Dbe[i][j] for j in range(p)] for i in range(n)]
        out["Xs"].append(X)
        out["Rs"].append(R)
        out["Ds"].append(D)
        out["alphas"].append(alpha)
        out["betas"].append(beta)
    return out
