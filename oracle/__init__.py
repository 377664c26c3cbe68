"""Oracle for cooperative conjugate gradient: plain FP64 CPU code.

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the library under
``paper_1204_0069_amd`` never does, and the two share no code.

The arithmetic lives in ``ccg_oracle.c`` (plain loops, column-major).  This module
only builds it with gcc, loads it with ctypes and marshals numpy arrays.  The source
is built twice: ``libccg_oracle.so`` computes in FP64 (double), the oracle proper;
``libccg_oracle_ld.so`` runs the same code with every internal value in x86 80-bit
extended precision (``long double``, 11 more significand bits), as a reference for
how far an FP64 trajectory of the method has drifted from the method's own
trajectory (``extended()``); ``libccg_oracle_omp.so`` is the FP64 oracle with its
products with A split by rows over OpenMP threads, bit-identical to the first, for
timing it on all host cores (``all_cores()``).  All take and return FP64 arrays.

Entry points
------------
``ccg(A, b, X0, tol, maxit, tau)``
    Alg. 2 of the paper (cooperative CG, Sec. 3.2) with the Table 1 residual
    recurrence, the Alg. 3 rank step (mcCG) and the Alg. 4 minimum-residual stop
    test, in the sign convention R = B - A X.  Returns the final agents X
    (n x p), the per-step alpha/beta trace if asked, the final R and D if asked,
    and an info dict.
``residual(A, b, X)``
    B - A X in FP64 with plain loops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccg_oracle.c")
_LIB = os.path.join(_HERE, "libccg_oracle.so")
_LIB_LD = os.path.join(_HERE, "libccg_oracle_ld.so")
_LIB_OMP = os.path.join(_HERE, "libccg_oracle_omp.so")

# gcc flags: baseline x86-64 (the library built here also runs on other hosts),
# no FMA contraction so every product and sum rounds as written.
GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off", "-fno-fast-math"]

ORC_STATUS = {0: "ok", 1: "not_converged", -1: "err_arg", -2: "err_nonfinite",
              -3: "err_not_spd", -5: "err_nomem"}


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("restarts", ctypes.c_int), ("p_final", ctypes.c_int),
                ("best_agent", ctypes.c_int), ("deflations", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("rel_res_max", ctypes.c_double),
                ("reinflations", ctypes.c_int)]


def _build_one(path: str, extra, force: bool) -> None:
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, *extra, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile ccg_oracle.c into libccg_oracle.so (FP64) and libccg_oracle_ld.so
    (80-bit extended) next to it (gcc)."""
    _build_one(_LIB, [], force)
    _build_one(_LIB_LD, ["-DORC_REAL=long double"], force)
    _build_one(_LIB_OMP, ["-fopenmp", "-DORC_ROWS=1024"], force)
    return _LIB


_lib = None
_lib_ld = None
_lib_omp = None


def bind(path: str):
    """Load a compiled oracle library from ``path`` and declare its signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_ccg.restype = ctypes.c_int
    lib.oracle_ccg.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp, dp,
                               ctypes.c_int, ctypes.c_double, ctypes.c_int,
                               ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int,
                               ctypes.POINTER(_Info)]
    lib.oracle_splitmix64.restype = None
    lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_residual.restype = ctypes.c_int
    lib.oracle_residual.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp,
                                    dp, ctypes.c_int, dp]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = bind(_LIB)
    return _lib


def all_cores():
    """The FP64 oracle built with OpenMP: the products with A split by rows over the
    threads (OMP_NUM_THREADS), with the same bits as the one-thread build (pass as
    ``lib``).  For timing the oracle on every host core."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_omp = bind(_LIB_OMP)
    return _lib_omp


def extended():
    """The oracle built with 80-bit extended internal arithmetic (pass as ``lib``)."""
    global _lib_ld
    if _lib_ld is None:
        if not os.path.exists(_LIB_LD) or os.path.getmtime(_LIB_LD) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_ld = bind(_LIB_LD)
    return _lib_ld


def _ptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _colmajor(A):
    return np.asfortranarray(np.asarray(A, dtype=np.float64))


def ccg(A, b, X0, tol: float, maxit: int, tau: float = 1e-14, trace_k: int = 0,
        want_rd: bool = False, lib=None, reinflate_max: int = 0) -> dict:
    """Run the oracle cCG.  A (n x n), b (n,), X0 (n x p) are numpy arrays.

    tol == 0 runs exactly ``maxit`` steps with no stop test.  reinflate_max > 0 lets
    up to that many rank drops re-inflate the dropped agents (see oracle_ccg in the C
    source) instead of going on with fewer.  Returns a dict with
    X, info fields, and (if asked) alphas/betas of shape (trace_k, p, p) indexed
    [step, row, col] and the final R, D (n x p).  ``lib`` selects another build of
    the same source (see ``bind``).
    """
    lib = lib or _load()
    A = _colmajor(A)
    n = A.shape[0]
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    X = _colmajor(np.array(X0, dtype=np.float64, copy=True).reshape(n, -1))
    p = X.shape[1]
    ta = tb = None
    if trace_k > 0:
        ta = np.zeros(trace_k * p * p)
        tb = np.zeros(trace_k * p * p)
    Rout = Dout = None
    if want_rd:
        Rout = np.zeros(n * p)
        Dout = np.zeros(n * p)
    info = _Info()
    lib.oracle_ccg(n, p, _ptr(A), n, _ptr(b), _ptr(X), n, float(tol), int(maxit),
                   float(tau), int(trace_k), _ptr(ta), _ptr(tb), _ptr(Rout), _ptr(Dout),
                   int(reinflate_max), ctypes.byref(info))
    out = {"X": X, "status": info.status, "status_name": ORC_STATUS.get(info.status, "?"),
           "iters": info.iters, "restarts": info.restarts, "p_final": info.p_final,
           "best_agent": info.best_agent, "deflations": info.deflations,
           "reinflations": info.reinflations,
           "rel_res": info.rel_res, "rel_res_max": info.rel_res_max}
    if trace_k > 0:
        # stored column-major per step: element (r, c) at r + c*p
        out["alphas"] = ta.reshape(trace_k, p, p).transpose(0, 2, 1).copy()
        out["betas"] = tb.reshape(trace_k, p, p).transpose(0, 2, 1).copy()
    if want_rd:
        out["R"] = Rout.reshape(p, n).T.copy()
        out["D"] = Dout.reshape(p, n).T.copy()
    return out


def splitmix64(state: int, count: int) -> list:
    """The first ``count`` outputs of the oracle's SplitMix64 generator from ``state``."""
    lib = _load()
    out = (ctypes.c_uint64 * count)()
    lib.oracle_splitmix64(ctypes.c_uint64(state), int(count), out)
    return [int(v) for v in out]


def residual(A, b, X) -> np.ndarray:
    """B - A X (n x p) in plain FP64 loops."""
    lib = _load()
    A = _colmajor(A)
    n = A.shape[0]
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    X = _colmajor(np.asarray(X, dtype=np.float64).reshape(n, -1))
    p = X.shape[1]
    T = np.zeros(n * p)
    st = lib.oracle_residual(n, p, _ptr(A), n, _ptr(b), _ptr(X), n, _ptr(T))
    if st != 0:
        raise ValueError(f"oracle_residual: status {st}")
    return T.reshape(p, n).T.copy()
