"""Seeded synthetic inputs for cooperative CG: dense SPD systems and start blocks.

This module is shared by the tests, the benchmark and the oracle side.  It holds
no arithmetic of the solver: it only draws random matrices and vectors.

Recipes (all FP64):

* ``spd_spectrum(n, kappa, seed)``: A = Q diag(lam) Q^T, Q from the QR factorisation
  of a seeded N(0,1) n x n matrix with the signs of R's diagonal folded into Q (a
  Haar-distributed orthogonal matrix), lam log-uniform in [1, kappa] with
  lam_min = 1 and lam_max = kappa forced so the condition number is exact, then
  A = (A + A^T)/2 so that A is exactly symmetric.  ``lam_dist="uniform"`` gives the
  paper's own test matrices (eigenvalues uniform in [1, kappa], Sec. 5).
* ``spd_gram(n, kappa, seed)``: A = M^T M / n + sigma I with M ~ N(0,1), sigma chosen
  from the largest eigenvalue of M^T M / n (power iteration) so that
  cond(A) ~= kappa (the smallest eigenvalue of M^T M / n, O(1/n^2), is neglected).
* ``normal_block(n, p, seed)``: N(0,1) entries; ``uniform_block(n, p, seed, lo, hi)``:
  uniform entries (the paper's right-hand sides and starting points use [-10, 10]).

Generation runs on the CPU with numpy (``device="cpu"``) or on a GPU with torch
(``device="cuda"``); the bytes then feed both the library and the oracle.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

BASE_SEED = 1204


def item_seed(tag: str, index: int = 0, base: int = BASE_SEED) -> int:
    """Deterministic per-item seed from a config tag and an index."""
    h = hashlib.sha256(f"{base}:{tag}:{index}".encode()).digest()
    return int.from_bytes(h[:8], "little") & ((1 << 63) - 1)


def _eigs(rng, n, kappa, lam_dist):
    if n == 1:
        return np.ones(1)
    if lam_dist == "loguniform":
        lam = np.exp(rng.uniform(0.0, math.log(kappa), n))
    elif lam_dist == "uniform":
        lam = rng.uniform(1.0, kappa, n)
    else:
        raise ValueError(lam_dist)
    lam[0] = 1.0
    lam[-1] = kappa
    return lam


def spd_spectrum(n: int, kappa: float, seed: int, lam_dist: str = "loguniform",
                 device: str = "cpu"):
    """A = Q diag(lam) Q^T (see module docstring).  numpy array on cpu, torch tensor on cuda."""
    if device == "cpu":
        rng = np.random.default_rng(seed)
        M = rng.standard_normal((n, n))
        lam = _eigs(rng, n, kappa, lam_dist)
        Q, Rq = np.linalg.qr(M)
        Q = Q * np.sign(np.diag(Rq))
        A = (Q * lam) @ Q.T
        return (A + A.T) * 0.5
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    M = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
    rng = np.random.default_rng(seed)
    lam = torch.from_numpy(_eigs(rng, n, kappa, lam_dist)).to(device)
    Q, Rq = torch.linalg.qr(M)
    Q = Q * torch.sign(torch.diagonal(Rq))
    del M, Rq
    A = (Q * lam) @ Q.T.contiguous()
    del Q
    A = (A + A.T.contiguous()) * 0.5
    return A


def spd_gram(n: int, kappa: float, seed: int, device: str = "cpu", power_iters: int = 60):
    """A = M^T M / n + sigma I with sigma = lam_max(M^T M/n) / (kappa - 1)."""
    if device == "cpu":
        rng = np.random.default_rng(seed)
        M = rng.standard_normal((n, n))
        A = (M.T @ M) / n
        v = rng.standard_normal(n)
        for _ in range(power_iters):
            v = A @ v
            v /= np.linalg.norm(v)
        lmax = float(v @ (A @ v))
        sigma = lmax / (kappa - 1.0)
        A[np.diag_indices(n)] += sigma
        return (A + A.T) * 0.5
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    M = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
    A = (M.T.contiguous() @ M) / n
    del M
    v = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    for _ in range(power_iters):
        v = A @ v
        v /= torch.linalg.norm(v)
    lmax = float(v @ (A @ v))
    sigma = lmax / (kappa - 1.0)
    A.diagonal().add_(sigma)
    A = (A + A.T.contiguous()) * 0.5
    return A


def normal_block(n: int, p: int, seed: int) -> np.ndarray:
    """n x p block of N(0,1) entries (p == 0 gives a length-n vector)."""
    rng = np.random.default_rng(seed)
    if p == 0:
        return rng.standard_normal(n)
    return rng.standard_normal((n, p))


def uniform_block(n: int, p: int, seed: int, lo: float = -10.0, hi: float = 10.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if p == 0:
        return rng.uniform(lo, hi, n)
    return rng.uniform(lo, hi, (n, p))


# ---------------------------------------------------------------- named workloads

def small_system(n: int = 256, p: int = 3, kappa: float = 1e3, seed: int = BASE_SEED):
    """n=256, p=3, log-uniform spectrum in [1, 1e3], b and X0 ~ N(0,1) (CPU)."""
    A = spd_spectrum(n, kappa, item_seed("A", seed, base=n))
    b = normal_block(n, 0, item_seed("b", seed, base=n))
    X0 = normal_block(n, p, item_seed("X0", seed, base=n))
    return A, b, X0


def system(n: int, p: int, kappa: float, seed: int = BASE_SEED, device: str = "cpu",
           kind: str = "spectrum"):
    """A seeded system of any size.  kind: 'spectrum' (Q diag Q^T), 'gram' (M^T M/n + sI),
    or 'paper' (uniform spectrum, b and X0 uniform in [-10, 10])."""
    if kind == "spectrum":
        A = spd_spectrum(n, kappa, item_seed("A", seed, base=n), device=device)
        b = normal_block(n, 0, item_seed("b", seed, base=n))
        X0 = normal_block(n, p, item_seed("X0", seed, base=n))
    elif kind == "gram":
        A = spd_gram(n, kappa, item_seed("G", seed, base=n), device=device)
        b = normal_block(n, 0, item_seed("b", seed, base=n))
        X0 = normal_block(n, p, item_seed("X0", seed, base=n))
    elif kind == "paper":
        A = spd_spectrum(n, kappa, item_seed("P", seed, base=n), lam_dist="uniform",
                         device=device)
        b = uniform_block(n, 0, item_seed("pb", seed, base=n))
        X0 = uniform_block(n, p, item_seed("pX0", seed, base=n))
    else:
        raise ValueError(kind)
    return A, b, X0


def batch_specs(count: int = 1024, seed: int = BASE_SEED, n_lo: int = 64, n_hi: int = 4096,
                p_choices=(2, 4, 8), k_lo: float = 1e2, k_hi: float = 1e5):
    """Sizes for a batch of independent systems: n log-uniform in [n_lo, n_hi],
    p uniform over p_choices, kappa log-uniform in [k_lo, k_hi]."""
    rng = np.random.default_rng(item_seed("batch", seed))
    ns = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(int)
    ps = rng.choice(np.asarray(p_choices), count)
    ks = np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), count))
    return [dict(n=int(n), p=int(min(p, n)), kappa=float(k), seed=int(item_seed("bi", i, seed)))
            for i, (n, p, k) in enumerate(zip(ns, ps, ks))]


def serve_specs(count: int, rate: float, seed: int = BASE_SEED, n_lo: int = 128,
                n_hi: int = 16384, p: int = 4, k_lo: float = 1e2, k_hi: float = 1e6,
                precisions=("fp64", "fp32", "bf16x2")):
    """A Poisson arrival stream: exponential inter-arrival times at ``rate`` per second,
    n log-uniform, kappa log-uniform, precision uniform over ``precisions``."""
    rng = np.random.default_rng(item_seed("serve", seed))
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(int)
    ks = np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), count))
    pr = rng.integers(0, len(precisions), count)
    return [dict(t=float(ti), n=int(n), p=p, kappa=float(k), prec=precisions[int(q)],
                 seed=int(item_seed("si", i, seed)))
            for i, (ti, n, k, q) in enumerate(zip(t, ns, ks, pr))]


def integer_system(n: int, p: int, seed: int, m_lo: int = -3, m_hi: int = 3,
                   v_lo: int = -5, v_hi: int = 5):
    """Tiny exactly-representable SPD system: A = M^T M + I with integer M, integer b
    and X0 (lists of Python ints, for exact-arithmetic checks)."""
    rng = np.random.default_rng(seed)
    M = rng.integers(m_lo, m_hi + 1, (n, n))
    A = M.T @ M + np.eye(n, dtype=np.int64)
    b = rng.integers(v_lo, v_hi + 1, n)
    X0 = rng.integers(v_lo, v_hi + 1, (n, p))
    return ([[int(v) for v in row] for row in A], [int(v) for v in b],
            [[int(v) for v in row] for row in X0])
