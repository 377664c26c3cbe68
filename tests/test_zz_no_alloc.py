"""ccg_solve_noalloc: the FP64 solve with its workspace in the library's device
scratch array (for callers that cannot allocate).  Checked through the C ABI against
ccg_solve on the same inputs, bit for bit, on two calls in a row (the second smaller,
so that stale padded rows, tickets and state of the first would show), and for
allocating nothing on the device and rejecting what it cannot serve."""
import ctypes

import numpy as np
import pytest
import torch

import ccg_inputs as ci

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _both(ctx, A, b, X0, tol, maxit, **opts):
    """(X, info) of ccg_solve and of ccg_solve_noalloc on the same inputs."""
    from paper_1204_0069_amd import CCG_NO_GRAPH
    Xs, is_ = ctx.solve(A, b, X0, tol, maxit, raise_on_error=False, flags=CCG_NO_GRAPH, **opts)
    Xn = X0.t().contiguous().clone()          # p x n: the column-major agents
    inn = ctx.solve_noalloc(A, b, Xn, tol, maxit, raise_on_error=False, **opts)
    return Xs, is_, Xn.t(), inn


def _same(Xs, is_, Xn, inn):
    assert inn["status"] == is_["status"]
    for k in ("iters", "restarts", "p_final", "best_agent", "deflations", "rel_res", "rel_res_max", "bytes_A"):
        assert inn[k] == is_[k], (k, inn[k], is_[k])
    assert torch.equal(Xn, Xs)


def test_noalloc_matches_solve_on_two_calls(gpu_ctx):
    # first larger systems (P = 32 and P = 16 on the matrix-core update launches,
    # then P = 8), then a smaller one in the same scratch
    for n, p, kappa, seed in [(1500, 20, 1e2, 74), (1800, 12, 1e2, 75), (2000, 8, 1e3, 71), (700, 3, 1e3, 72)]:
        print(f"case noalloc n={n} p={p}", flush=True)
        A, b, X0 = ci.system(n, p, kappa, seed=seed)
        Xs, is_, Xn, inn = _both(gpu_ctx, _t(A), _t(b), _t(X0), 1e-10, 20000)
        assert is_["status"] == 0 and is_["iters"] > 0
        _same(Xs, is_, Xn, inn)
        # and the graph-launched solve gives the same result
        Xg, ig = gpu_ctx.solve(_t(A), _t(b), _t(X0), 1e-10, 20000)
        assert ig["iters"] == inn["iters"] and torch.equal(Xg, Xn)


def test_noalloc_allocates_nothing():
    """A fresh context: after one warm-up call (the kernels loaded), a call whose
    workspace is about 29 MB leaves the device's free memory unchanged, and matches
    ccg_solve (which allocates that workspace) bit for bit."""
    from paper_1204_0069_amd import Context
    ctx = Context(0)
    try:
        A, b, X0 = ci.system(300, 16, 1e2, seed=73)
        Xw = _t(X0).t().contiguous().clone()
        ctx.solve_noalloc(_t(A), _t(b), Xw, 1e-10, 50)
        n, p = 16384, 16
        A = ci.spd_spectrum(n, 1e3, ci.item_seed("A", 74, base=n), device=DEV)
        b = _t(ci.normal_block(n, 0, 75))
        X0 = _t(ci.normal_block(n, p, 76))
        Xn = X0.t().contiguous().clone()
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        inn = ctx.solve_noalloc(A, b, Xn, 1e-10, 3, raise_on_error=False)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        print(f"free memory {free0} -> {free1}", flush=True)
        assert inn["status"] == 1 and inn["iters"] == 3
        assert abs(free1 - free0) < (4 << 20)
        Xs, is_ = ctx.solve(A, b, X0, 1e-10, 3, raise_on_error=False)
        _same(Xs, is_, Xn.t(), inn)
    finally:
        ctx.close()


def test_noalloc_rejects_what_it_cannot_serve(gpu_ctx):
    from paper_1204_0069_amd import CCG_HOST_PTRS, CCG_SYM_AD
    lib, h = gpu_ctx.lib, gpu_ctx.h
    A, b, X0 = ci.system(64, 2, 10.0, seed=77)
    At, bt = _t(A), _t(b)
    Xn = _t(X0).t().contiguous().clone()
    for opts in ({"prec": "fp32"}, {"flags": CCG_HOST_PTRS}, {"flags": CCG_SYM_AD}):
        info = gpu_ctx.solve_noalloc(At, bt, Xn, 1e-10, 100, raise_on_error=False, **opts)
        assert info["status"] == -1, opts
    from paper_1204_0069_amd.ccg import Info, make_opts
    o = make_opts()
    info = Info()
    # odd leading dimension: columns not 16-byte aligned
    big = torch.zeros(65, 65, dtype=torch.float64, device=DEV)
    st = lib.ccg_solve_noalloc(h, 64, 2, big.data_ptr(), 65, bt.data_ptr(), Xn.data_ptr(), 64, 1e-10, 100,
                               ctypes.byref(o), ctypes.byref(info))
    assert st == -1
    # a workspace beyond the scratch array: rejected before anything is launched (the
    # pointers are never read)
    st = lib.ccg_solve_noalloc(h, 70000, 16, At.data_ptr(), 70000, bt.data_ptr(), Xn.data_ptr(), 70000, 1e-10,
                               100, ctypes.byref(o), ctypes.byref(info))
    assert st == -5
    assert b"scratch" in lib.ccg_last_error(h)
    # the context still works
    Xn2 = _t(X0).t().contiguous().clone()
    info = gpu_ctx.solve_noalloc(At, bt, Xn2, 1e-10, 100)
    assert info["status"] == 0
