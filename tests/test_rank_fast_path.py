"""The keep-all test of the rank step (Alg. 3) that the A.D launch's last workgroup
runs before the greedy rule.

For the diagonally scaled G (unit diagonal, positive semidefinite) the greedy pivoted
Cholesky factorisation takes its pivots in non-increasing order (an elimination only
lowers the remaining diagonal, and the largest is taken next), and its last pivot is
the Schur complement of the index taken last, 1 / (G^-1)_ll.  Every pivot is therefore
at least 1 / max_l (G^-1)_ll, and when that bound exceeds 2 tau the greedy rule keeps
every agent.  The kernel first tests the determinant of the scaled G (a weaker bound:
each 1 / (G^-1)_ll is at least the determinant) and, when that fails, forms the bound
from the natural-order Cholesky factor (lane l solves L y = e_l, (G^-1)_ll = G_ll ||y||^2
for the unscaled G).  Here a plain
greedy factorisation, written from the rule (largest remaining pivot first, ties to
the lowest index, stop at a pivot <= tau), checks both facts and the decision on
random and nearly singular matrices around tau = 1e-14."""
import numpy as np
import pytest

TAU = 1e-14


def greedy_pivots(G, tau):
    S = np.array(G, dtype=np.float64)
    left = list(range(S.shape[0]))
    piv = []
    while left:
        i = max(left, key=lambda k: (S[k, k], -k))
        d = S[i, i]
        if not d > tau:
            break
        piv.append(d)
        left.remove(i)
        if left:
            col = S[left, i] / np.sqrt(d)
            S[np.ix_(left, left)] -= np.outer(col, col)
    return piv, not left


def keep_all_bound(G):
    """The kernel's estimate: natural-order Cholesky of the unscaled G, then
    G_ll ||L^-1 e_l||^2 per l; returns 1 / max_l, or 0 when the factor fails."""
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return 0.0
    m = G.shape[0]
    q = []
    for l in range(m):
        y = np.zeros(m)
        for k in range(m):
            t = (1.0 if k == l else 0.0) - L[k, :k] @ y[:k]
            y[k] = t / L[k, k]
        q.append(G[l, l] * (y @ y))
    mq = max(q)
    return 1.0 / mq if np.isfinite(mq) and mq > 0 else 0.0


def scaled(G):
    s = 1.0 / np.sqrt(np.diag(G))
    return G * s[:, None] * s[None, :]


def gram(rng, m, smin, scale_spread):
    """G = D^T A D-like: B^T B with singular values from 1 down to smin, columns
    scaled by factors spread over scale_spread decades (the scaling is undone by the
    rank step's diagonal scaling, not by the kernel's factor)."""
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sv = np.logspace(0, np.log10(smin), m)
    B = U @ np.diag(sv) @ V.T
    c = 10.0 ** rng.uniform(-scale_spread, scale_spread, m)
    B = B * c[None, :]
    return B.T @ B


@pytest.mark.parametrize("m", [2, 4, 8, 16, 32])
def test_greedy_pivots_never_increase_and_end_at_the_schur_complement(m):
    rng = np.random.default_rng(1000 + m)
    for _ in range(40):
        G = scaled(gram(rng, m, 10.0 ** rng.uniform(-4, 0), 3))
        piv, full = greedy_pivots(G, 0.0)
        assert all(b <= a for a, b in zip(piv, piv[1:]))
        if full:
            Ginv = np.linalg.inv(G)
            # the last pivot is 1 / (G^-1)_ll of some l, and no smaller than the bound
            last = piv[-1]
            assert min(abs(last * Ginv[l, l] - 1.0) for l in range(m)) < 1e-6
            assert last >= (1.0 - 1e-6) / np.max(np.diag(Ginv))


@pytest.mark.parametrize("m", [2, 3, 8, 16, 32])
def test_the_keep_all_test_never_keeps_what_the_greedy_rule_drops(m):
    rng = np.random.default_rng(2000 + m)
    kept_fast = dropped = 0
    for _ in range(300):
        # smallest singular value of B around sqrt(tau): pivots straddle tau
        G = gram(rng, m, 10.0 ** rng.uniform(-8.5, -5.5), 4)
        piv, full = greedy_pivots(scaled(G), TAU)
        if keep_all_bound(G) * 1.0 > 2.0 * TAU:
            kept_fast += 1
            assert full, (m, piv[-3:])
        if not full:
            dropped += 1
    # the sample reaches both sides of the threshold
    assert kept_fast > 0 and dropped > 0


def test_the_bound_is_never_below_the_determinant():
    """The earlier test (det of the scaled G > 2 tau) is implied by the new one: for a
    unit-diagonal PD matrix 1 / (G^-1)_ll = det G / det G_(-l) >= det G."""
    rng = np.random.default_rng(7)
    for m in (2, 4, 8):
        for _ in range(50):
            G = gram(rng, m, 10.0 ** rng.uniform(-4, 0), 2)
            Gs = scaled(G)
            assert keep_all_bound(G) >= np.linalg.det(Gs) * (1.0 - 1e-9)
