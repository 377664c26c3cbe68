"""GPU tests of the mixed-precision modes (FP32 / BF16x2 A in FP64 refinement).

* The low-precision copies of A are integer-exact work: compared bit for bit with
  the conversion oracle (oracle/lowprec.py) through ccg_convert_matrix.
* A refined solve has no oracle trajectory (its iterates differ from any FP64 run
  by design), so it is held to what fixes the answer: the explicit FP64 residual of
  the best agent, recomputed by the oracle, is <= tol, and that agent is within
  2 * cond(A) * tol of the direct solution (relative).
"""
import numpy as np
import pytest
import torch

import ccg_inputs as ci
import oracle
from oracle import lowprec as lp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _wide_matrix(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) * np.exp(rng.uniform(-30, 30, (n, n)))
    M[0, 0] = 0.0
    M[1 % n, 0] = 1.0 + 0.5 / 128.0          # a BF16 tie
    return M


@pytest.mark.parametrize("n", [1, 37, 256, 1000])
def test_fp32_copy_is_bit_exact(gpu_ctx, n):
    print(f"case convert fp32 n={n}", flush=True)
    M = _wide_matrix(n, n)
    got = gpu_ctx.convert_matrix(_t(M), "fp32").cpu().numpy()
    want = lp.to_f32(M)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("n", [1, 37, 256, 1000])
def test_bf16x2_copy_is_bit_exact(gpu_ctx, n):
    print(f"case convert bf16x2 n={n}", flush=True)
    M = _wide_matrix(n, 100 + n)
    hi, lo = gpu_ctx.convert_matrix(_t(M), "bf16x2")
    whi, wlo = lp.to_bf16x2(M)
    assert np.array_equal(hi.cpu().numpy().view(np.uint16), lp.bf16_bits(whi))
    assert np.array_equal(lo.cpu().numpy().view(np.uint16), lp.bf16_bits(wlo))


def _residual_noise(A, b, x):
    """Bound on the rounding of a computed relative residual ||b - A x|| / ||b||:
    each entry of b - A x carries at most n * eps * (|b| + |A| |x|) (standard
    summation bound), for either summation order."""
    n = A.shape[0]
    scale = np.abs(b) + np.abs(A) @ np.abs(x)
    return 2.0 * n * 1.11e-16 * np.linalg.norm(scale) / np.linalg.norm(b)


def _check_refined(A, b, X, info, tol, kappa):
    Xg = X.cpu().numpy()
    T = oracle.residual(A, b, Xg)
    rel = np.linalg.norm(T, axis=0) / np.linalg.norm(b)
    assert info["status"] == 0, info
    assert rel.min() <= tol, (rel.min(), info)
    j = info["best_agent"]
    noise = _residual_noise(A, b, Xg[:, j])
    # the library's explicit residual and the oracle's agree up to rounding; the
    # best agent is a true argmin up to the same rounding
    assert abs(info["rel_res"] - rel[j]) <= 1e-3 * rel[j] + noise, (info["rel_res"], rel[j], noise)
    assert rel[j] <= rel.min() + 2 * noise
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(Xg[:, j] - xs) <= 2 * kappa * tol * np.linalg.norm(xs)
    assert info["refinements"] >= 1 and info["iters"] >= 1


FP32_CASES = [(256, 3, 1e3), (1000, 4, 1e3), (777, 2, 1e2), (640, 16, 1e2), (300, 1, 1e3),
              (2085, 8, 1e4)]
BF16_CASES = [(256, 3, 1e3), (1000, 4, 1e3), (777, 2, 1e2), (640, 16, 1e2), (300, 1, 1e2)]


@pytest.mark.parametrize("n,p,kappa", FP32_CASES)
def test_fp32_refined_solve(gpu_ctx, n, p, kappa):
    print(f"case solve fp32 n={n} p={p} kappa={kappa}", flush=True)
    A, b, X0 = ci.system(n, p, kappa, seed=303)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32")
    _check_refined(A, b, X, info, 1e-10, kappa)


@pytest.mark.parametrize("n,p,kappa", BF16_CASES)
def test_bf16x2_refined_solve(gpu_ctx, n, p, kappa):
    print(f"case solve bf16x2 n={n} p={p} kappa={kappa}", flush=True)
    A, b, X0 = ci.system(n, p, kappa, seed=404)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="bf16x2")
    _check_refined(A, b, X, info, 1e-10, kappa)


def test_refined_solve_is_deterministic(gpu_ctx):
    A, b, X0 = ci.system(900, 4, 1e3, seed=9)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32")
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32")
    assert i1["iters"] == i2["iters"] and i1["refinements"] == i2["refinements"]
    assert torch.equal(X1, X2)


def test_refined_graph_and_direct_launch_agree(gpu_ctx):
    from paper_1204_0069_amd import CCG_NO_GRAPH
    A, b, X0 = ci.system(700, 8, 1e3, seed=10)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="bf16x2")
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="bf16x2", flags=CCG_NO_GRAPH)
    assert i1["iters"] == i2["iters"]
    assert torch.equal(X1, X2)


def test_refined_timed_launches_agree(gpu_ctx):
    """Timing the inner A.D launches (every round, or every 4th) leaves the refined
    solve bit for bit the same."""
    from paper_1204_0069_amd import CCG_PROFILE, CCG_PROFILE_SAMPLED
    A, b, X0 = ci.system(900, 4, 1e3, seed=11)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32")
    gpu_ctx.kernel_time(reset=True)
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32", flags=CCG_PROFILE_SAMPLED)
    _, n_s = gpu_ctx.kernel_time(reset=True)
    X3, i3 = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32", flags=CCG_PROFILE)
    _, n_all = gpu_ctx.kernel_time(reset=True)
    assert i1["iters"] == i2["iters"] == i3["iters"]
    assert torch.equal(X1, X2) and torch.equal(X1, X3)
    assert 0 < n_s < n_all


def test_refinement_limits(gpu_ctx):
    A, b, X0 = ci.system(500, 4, 1e3, seed=12)
    # one outer step cannot reach 1e-10 with an inner tolerance of 1e-4
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec="fp32", max_refine=1,
                            raise_on_error=False)
    assert info["status"] == 1 and info["refinements"] == 1
    # a total step budget stops the refinement too
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 30, prec="fp32", raise_on_error=False)
    assert info["status"] == 1 and info["iters"] <= 30


def test_full_size_fp32_solve(gpu_ctx):
    n, p, kappa = 8192, 8, 1e4
    print("case full-size fp32 n=8192 p=8", flush=True)
    A = ci.spd_spectrum(n, kappa, ci.item_seed("A", ci.BASE_SEED, base=n), device=DEV)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", ci.BASE_SEED, base=n)), device=DEV)
    X0 = torch.as_tensor(ci.normal_block(n, p, ci.item_seed("X0", ci.BASE_SEED, base=n)), device=DEV)
    X, info = gpu_ctx.solve(A, b, X0, 1e-10, 100000, prec="fp32")
    assert info["status"] == 0, info
    # explicit residual of every agent with torch's own product (rocBLAS)
    T = b[:, None] - A @ X
    rel = (torch.linalg.norm(T, dim=0) / torch.linalg.norm(b)).cpu().numpy()
    assert rel.min() <= 1e-10
    j = info["best_agent"]
    x = X[:, j]
    noise = float(2.0 * n * 1.11e-16 * torch.linalg.norm(b.abs() + A.abs() @ x.abs()) / torch.linalg.norm(b))
    assert abs(info["rel_res"] - rel[j]) <= 1e-3 * rel[j] + noise


def test_escalation_after_breakdown(gpu_ctx):
    """At cond(A) = 1e8 the BF16x2 copy of A (about 2^-17 relative error per element)
    is too coarse for its refinement to progress; with CCG_ESCALATE the solve goes on
    from its agents in a wider precision, meets the target, reports the precision it
    ended in and totals over every stage.  (At cond 1e10 the FP64 stage alone takes
    anywhere from 2e4 to over 1e5 block steps, depending on rounding, in the oracle as
    on the GPU, which makes a step limit a coin toss.)"""
    from paper_1204_0069_amd import CCG_ESCALATE
    n, p, kappa, tol = 128, 4, 1e8, 1e-5
    A, b, X0 = ci.system(n, p, kappa, seed=505)
    X1, i1 = gpu_ctx.solve(_t(A), _t(b), _t(X0), tol, 100000, prec="bf16x2", raise_on_error=False)
    assert i1["status"] != 0 and i1["prec_final"] == 2, i1
    X2, i2 = gpu_ctx.solve(_t(A), _t(b), _t(X0), tol, 100000, prec="bf16x2", flags=CCG_ESCALATE)
    assert i2["status"] == 0 and i2["prec_final"] in (0, 1), i2
    T = oracle.residual(A, b, X2.cpu().numpy())
    assert (np.linalg.norm(T, axis=0) / np.linalg.norm(b)).min() <= 1.01 * tol
    assert i2["iters"] > i1["iters"] and i2["bytes_A"] > i1["bytes_A"]


@pytest.fixture(scope="module")
def c3_system():
    """The n = 32768, p = 8 workload of the mixed-precision modes (A = M^T M / n + sigma I,
    cond 1e3, built on the device)."""
    n, p = 32768, 8
    A = ci.spd_gram(n, 1e3, ci.item_seed("C3", 1204, base=n), device=DEV)
    b = torch.as_tensor(ci.normal_block(n, 0, ci.item_seed("b", 1204, base=n)), device=DEV)
    X0 = torch.as_tensor(ci.normal_block(n, p, ci.item_seed("X0", 1204, base=n)), device=DEV)
    yield A, b, X0
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_full_size_n32768_refined_solve(gpu_ctx, c3_system, prec):
    """At n = 32768 (4 GiB as BF16 hi + lo planes, 8 GiB in FP64) the oracle cannot run a
    solve; what holds at any size is checked instead: the low-precision copy is the
    oracle's conversion, bit for bit, on sampled columns; the explicit FP64 residual of
    the best agent (torch's own product) meets tol and matches the reported one; and
    sampled rows of that residual, summed in FP64 on the host, agree with it."""
    A, b, X0 = c3_system
    n = A.shape[0]
    print(f"case full-size {prec} n={n} p=8", flush=True)
    rng = np.random.default_rng(32768)
    cols = np.sort(rng.choice(n, 4, replace=False))
    Ac = A[:, cols].cpu().numpy()          # columns of the symmetric A, also its rows
    # (the copy keeps A's element order; A is symmetric, so columns are rows too)
    if prec == "fp32":
        lowA = gpu_ctx.convert_matrix(A, "fp32")
        got = lowA[:, cols].cpu().numpy()
        del lowA
        assert np.array_equal(got.view(np.uint32), lp.to_f32(Ac).view(np.uint32))
    else:
        hi, lo = gpu_ctx.convert_matrix(A, "bf16x2")
        ghi, glo = hi[:, cols].cpu().numpy(), lo[:, cols].cpu().numpy()
        del hi, lo
        whi, wlo = lp.to_bf16x2(Ac)
        assert np.array_equal(ghi.view(np.uint16), lp.bf16_bits(whi))
        assert np.array_equal(glo.view(np.uint16), lp.bf16_bits(wlo))
    torch.cuda.empty_cache()
    X, info = gpu_ctx.solve(A, b, X0, 1e-10, 100000, prec=prec)
    assert info["status"] == 0, info
    T = b[:, None] - A @ X
    rel = (torch.linalg.norm(T, dim=0) / torch.linalg.norm(b)).cpu().numpy()
    j = info["best_agent"]
    assert rel[j] <= 1e-10 and abs(info["rel_res"] - rel[j]) <= 1e-3 * rel[j] + 1e-14
    xj = X[:, j].cpu().numpy()
    rows = np.sort(rng.choice(n, 8, replace=False))
    Ar = A[rows, :].cpu().numpy()
    t_host = b.cpu().numpy()[rows] - Ar @ xj
    scale = np.abs(b.cpu().numpy()[rows]) + np.abs(Ar) @ np.abs(xj)
    assert np.all(np.abs(t_host - T[rows, j].cpu().numpy()) <= 2.0 * n * 1.11e-16 * scale)


# ------------- the FP32-operand matrix-core A.D tile (FP32 and BF16x2 A, P = 16)

# (cw, nw) shapes that run it: 16 or 32 AD rows per workgroup, 4 to 16 waves
MMA32_SHAPES = [(4, 4), (2, 8), (4, 8), (1, 16), (2, 16)]
# n below one chunk of 256 contraction indices (the guarded partial chunk only), several
# chunks with a ragged last one, p padded to 16


@pytest.mark.parametrize("shape", MMA32_SHAPES)
@pytest.mark.parametrize("n,p", [(200, 12), (1000, 16), (2085, 9)])
@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_matrix_core_ad_refined_solve(gpu_ctx, prec, n, p, shape):
    """Every matrix-core shape meets the explicit FP64 residual and the distance to the
    direct solution, and needs about as many block steps as the vector tile (2, 4): a
    wrong A.D product would cost the refinement loop far more steps or not converge."""
    cw, nw = shape
    print(f"case mma32 {prec} n={n} p={p} shape={shape}", flush=True)
    A, b, X0 = ci.system(n, p, 1e2, seed=505)
    X, info = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec=prec, ad_cw=cw, ad_nw=nw)
    _check_refined(A, b, X, info, 1e-10, 1e2)
    Xv, iv = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 100000, prec=prec, ad_cw=2, ad_nw=4)
    assert iv["status"] == 0
    assert info["iters"] <= 1.25 * iv["iters"] + 8, (info["iters"], iv["iters"])
