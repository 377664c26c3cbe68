"""Python binding of libccg.so (include/ccg.h): argument marshalling only.

Every step of the solve runs in the HIP kernels of the library; torch provides the
device buffers.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccg.so")

CCG_HOST_PTRS = 0x1
CCG_NO_GRAPH = 0x2
CCG_PROFILE = 0x4
CCG_PROFILE_SAMPLED = 0x10
CCG_ESCALATE = 0x8
CCG_SYM_AD = 0x20
CCG_REINFLATE = 0x40
CCG_NO_TIER = 0x80

PREC = {"fp64": 0, "fp32": 1, "bf16x2": 2}

STATUS = {0: "ok", 1: "not_converged", -1: "err_arg", -2: "err_nonfinite", -3: "err_not_spd",
          -4: "err_breakdown", -5: "err_nomem", -6: "err_device", -7: "pending", -8: "cancelled"}


class CcgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("inner_maxit", ctypes.c_int), ("max_refine", ctypes.c_int),
                ("rank_tau", ctypes.c_double), ("graph_k", ctypes.c_int),
                ("flags", ctypes.c_uint), ("max_reinflate", ctypes.c_int),
                ("ad_cw", ctypes.c_int), ("ad_nw", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("refinements", ctypes.c_int), ("restarts", ctypes.c_int),
                ("p_final", ctypes.c_int), ("best_agent", ctypes.c_int),
                ("deflations", ctypes.c_int), ("prec_final", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("rel_res_max", ctypes.c_double),
                ("seconds", ctypes.c_double), ("bytes_A", ctypes.c_double),
                ("reinflations", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("b", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("opts", Opts)]


_lib = None

# Entry points declared in include/ccg.h (kept in sync by tests/test_abi.py).
EXPORTS = ("ccg_create", "ccg_destroy", "ccg_last_error", "ccg_solve", "ccg_solve_noalloc", "ccg_debug_step",
           "ccg_solve_batched", "ccg_submit", "ccg_poll", "ccg_wait", "ccg_cancel",
           "ccg_convert_matrix", "ccg_tune_ad", "ccg_stream_probe", "ccg_kernel_time")


def load_library(path: str = LIB_PATH):
    """Load libccg.so (after torch, so both share one HIP runtime) and declare signatures."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1204_0069_amd.build`")
    lib = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.ccg_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t, vp]
    lib.ccg_create.restype = ctypes.c_int
    lib.ccg_destroy.argtypes = [vp]
    lib.ccg_destroy.restype = ctypes.c_int
    lib.ccg_last_error.argtypes = [vp]
    lib.ccg_last_error.restype = ctypes.c_char_p
    lib.ccg_solve.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, i64, vp, vp, i64,
                              ctypes.c_double, ctypes.c_int, ctypes.POINTER(Opts),
                              ctypes.POINTER(Info)]
    lib.ccg_solve.restype = ctypes.c_int
    lib.ccg_solve_noalloc.argtypes = lib.ccg_solve.argtypes
    lib.ccg_solve_noalloc.restype = ctypes.c_int
    lib.ccg_debug_step.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, i64, vp, vp, i64,
                                   ctypes.c_int, ctypes.POINTER(Opts), dp, dp, dp, dp]
    lib.ccg_debug_step.restype = ctypes.c_int
    lib.ccg_solve_batched.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Problem), ctypes.POINTER(Info)]
    lib.ccg_solve_batched.restype = ctypes.c_int
    lib.ccg_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_uint64)]
    lib.ccg_submit.restype = ctypes.c_int
    lib.ccg_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Info)]
    lib.ccg_poll.restype = ctypes.c_int
    lib.ccg_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Info)]
    lib.ccg_wait.restype = ctypes.c_int
    lib.ccg_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.ccg_cancel.restype = ctypes.c_int
    lib.ccg_convert_matrix.argtypes = [vp, ctypes.c_int, vp, i64, ctypes.c_int, vp, vp]
    lib.ccg_convert_matrix.restype = ctypes.c_int
    lib.ccg_tune_ad.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, dp]
    lib.ccg_tune_ad.restype = ctypes.c_int
    lib.ccg_stream_probe.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, dp]
    lib.ccg_stream_probe.restype = ctypes.c_int
    lib.ccg_kernel_time.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), dp, ctypes.c_int]
    lib.ccg_kernel_time.restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def _colmajor_matrix(A: torch.Tensor):
    """(pointer, lda) of a column-major view of A.  A row-major contiguous tensor is
    read as its own transpose, which is A itself for the symmetric matrices the method
    requires."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if A.dtype != torch.float64:
        raise TypeError("A must be float64")
    n = A.shape[0]
    if A.stride(0) == 1 and A.stride(1) >= n:
        return A.data_ptr(), A.stride(1), A
    if A.stride(1) == 1 and A.stride(0) >= n:
        return A.data_ptr(), A.stride(0), A
    Ac = A.contiguous()
    return Ac.data_ptr(), n, Ac


def make_opts(prec="fp64", inner_tol=0.0, inner_maxit=0, max_refine=0, rank_tau=0.0,
              graph_k=0, flags=0, max_reinflate=0, ad_cw=0, ad_nw=0) -> Opts:
    return Opts(PREC[prec] if isinstance(prec, str) else int(prec), float(inner_tol),
                int(inner_maxit), int(max_refine), float(rank_tau), int(graph_k), int(flags),
                int(max_reinflate), int(ad_cw), int(ad_nw))


def _problem(A: torch.Tensor, b: torch.Tensor, X0: torch.Tensor, tol: float, maxit: int, opts: dict):
    """(Problem, X, keep-alive list).  Tensors on the CPU are passed as host pointers
    (CCG_HOST_PTRS); X is the n x p result view."""
    host = A.device.type == "cpu"
    aptr, lda, Ak = _colmajor_matrix(A)
    n = A.shape[0]
    bb = b.reshape(-1).to(device=A.device, dtype=torch.float64).contiguous()
    Xt = X0.to(device=A.device, dtype=torch.float64).t().clone(memory_format=torch.contiguous_format)   # p x n = col-major n x p
    o = dict(opts)
    if host:
        o["flags"] = int(o.get("flags", 0)) | CCG_HOST_PTRS
    pr = Problem(n, Xt.shape[0], aptr, lda, bb.data_ptr(), Xt.data_ptr(), n, float(tol), int(maxit),
                 make_opts(**o))
    return pr, Xt.t(), [Ak, bb, Xt]


class Context:
    """A library context on one GPU (its own HIP stream, default priority)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.ccg_create(ctypes.byref(h), device, hbm_budget, None)
        if st != 0:
            raise CcgError(st, "ccg_create failed")
        self.h = h
        self._pending = {}

    def solve_batched(self, systems, raise_on_error: bool = False):
        """Solve many systems in shared launches.  systems: iterable of dicts with keys
        A, b, X0, tol, maxit and optional solver options.  Returns a list of (X, info)."""
        probs, outs, keep = [], [], []
        for sy in systems:
            sy = dict(sy)
            A, b, X0 = sy.pop("A"), sy.pop("b"), sy.pop("X0")
            tol, maxit = sy.pop("tol"), sy.pop("maxit")
            pr, X, k = _problem(A, b, X0, tol, maxit, sy)
            probs.append(pr)
            outs.append(X)
            keep.append(k)
        arr = (Problem * max(1, len(probs)))(*probs)
        infos = (Info * max(1, len(probs)))()
        torch.cuda.synchronize()
        st = self.lib.ccg_solve_batched(self.h, len(probs), arr, infos)
        if st < 0 and raise_on_error:
            raise self._err(st)
        del keep
        return [(outs[i], infos[i].as_dict()) for i in range(len(probs))]

    def submit(self, A: torch.Tensor, b: torch.Tensor, X0: torch.Tensor, tol: float, maxit: int,
               **opts) -> int:
        """Queue a system on the context's service; returns its ticket.  Its buffers are
        kept alive here until the ticket is polled or waited for."""
        pr, X, keep = _problem(A, b, X0, tol, maxit, opts)
        if A.device.type != "cpu":
            torch.cuda.synchronize(A.device)
        t = ctypes.c_uint64()
        st = self.lib.ccg_submit(self.h, ctypes.byref(pr), ctypes.byref(t))
        if st != 0:
            raise self._err(st)
        self._pending[t.value] = (X, keep)
        return t.value

    def _finish(self, ticket, st, info):
        X, _ = self._pending.pop(ticket, (None, None))
        d = info.as_dict()
        d["status"] = st
        d["status_name"] = STATUS.get(st, str(st))
        return X, d

    def poll(self, ticket: int):
        """(X, info) when the ticket has finished, else None."""
        info = Info()
        st = self.lib.ccg_poll(self.h, ticket, ctypes.byref(info))
        if st == -7:
            return None
        if st == -1 and ticket not in self._pending:
            raise self._err(st)
        return self._finish(ticket, st, info)

    def wait(self, ticket: int):
        """Block until the ticket finishes; returns (X, info)."""
        info = Info()
        st = self.lib.ccg_wait(self.h, ticket, ctypes.byref(info))
        if st == -1 and ticket not in self._pending:
            raise self._err(st)
        return self._finish(ticket, st, info)

    def cancel(self, ticket: int) -> None:
        st = self.lib.ccg_cancel(self.h, ticket)
        if st != 0:
            raise self._err(st)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ccg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st):
        return CcgError(st, self.lib.ccg_last_error(self.h).decode())

    def solve(self, A: torch.Tensor, b: torch.Tensor, X0: torch.Tensor, tol: float,
              maxit: int, raise_on_error: bool = True, **opts):
        """Solve A x = b with X0.shape[1] agents.  Returns (X, info dict); X is n x p."""
        aptr, lda, keep = _colmajor_matrix(A)
        n = A.shape[0]
        b = b.reshape(-1).to(device=A.device, dtype=torch.float64).contiguous()
        Xt = X0.to(device=A.device, dtype=torch.float64).t().clone(memory_format=torch.contiguous_format)   # p x n = col-major n x p
        p = Xt.shape[0]
        o = make_opts(**opts)
        info = Info()
        torch.cuda.synchronize(A.device)
        st = self.lib.ccg_solve(self.h, n, p, aptr, lda, b.data_ptr(), Xt.data_ptr(), n,
                                float(tol), int(maxit), ctypes.byref(o), ctypes.byref(info))
        if st < 0 and raise_on_error:
            raise self._err(st)
        del keep
        return Xt.t(), info.as_dict()

    def solve_noalloc(self, A: torch.Tensor, b: torch.Tensor, X: torch.Tensor, tol: float,
                      maxit: int, raise_on_error: bool = True, **opts):
        """ccg_solve_noalloc: the FP64 solve with its workspace in the library's device
        scratch array (no device allocation inside the call).  X is the p x n
        contiguous tensor that holds the column-major n x p agents: X0 in, the final
        agents out (updated in place).  A must be a contiguous float64 matrix with an
        even leading dimension.  Returns the info dict."""
        n = A.shape[0]
        if A.dtype != torch.float64 or not (A.is_contiguous() or A.t().is_contiguous()):
            raise ValueError("A must be a contiguous float64 matrix")
        if X.dim() != 2 or X.shape[1] != n or not X.is_contiguous() or X.dtype != torch.float64:
            raise ValueError("X must be a contiguous float64 p x n tensor (column-major n x p)")
        if b.dim() != 1 or b.shape[0] != n or not b.is_contiguous() or b.dtype != torch.float64:
            raise ValueError("b must be a contiguous float64 vector of length n")
        o = make_opts(**opts)
        info = Info()
        torch.cuda.synchronize(A.device)
        st = self.lib.ccg_solve_noalloc(self.h, n, X.shape[0], A.data_ptr(), n, b.data_ptr(),
                                        X.data_ptr(), n, float(tol), int(maxit), ctypes.byref(o),
                                        ctypes.byref(info))
        if st < 0 and raise_on_error:
            raise self._err(st)
        return info.as_dict()

    def debug_step(self, A: torch.Tensor, b: torch.Tensor, X0: torch.Tensor, ksteps: int,
                   rank_tau: float = 0.0, flags: int = 0, **opts):
        """Exactly ksteps FP64 block steps; returns dict of X, R, D (n x p, CPU float64)
        and alphas, betas (ksteps x p x p, [step, row, col])."""
        aptr, lda, keep = _colmajor_matrix(A)
        n = A.shape[0]
        b = b.reshape(-1).to(device=A.device, dtype=torch.float64).contiguous()
        Xt = X0.to(device=A.device, dtype=torch.float64).t().clone(memory_format=torch.contiguous_format)
        p = Xt.shape[0]
        R = torch.zeros(p, n, dtype=torch.float64, device=A.device)
        D = torch.zeros(p, n, dtype=torch.float64, device=A.device)
        al = (ctypes.c_double * max(1, ksteps * p * p))()
        be = (ctypes.c_double * max(1, ksteps * p * p))()
        o = make_opts(rank_tau=rank_tau, flags=flags, **opts)
        torch.cuda.synchronize(A.device)
        dptr = ctypes.POINTER(ctypes.c_double)
        st = self.lib.ccg_debug_step(self.h, n, p, aptr, lda, b.data_ptr(), Xt.data_ptr(), n,
                                     int(ksteps), ctypes.byref(o), al, be,
                                     ctypes.cast(R.data_ptr(), dptr), ctypes.cast(D.data_ptr(), dptr))
        if st < 0:
            raise self._err(st)
        del keep
        import numpy as np
        a = np.frombuffer(al, dtype=np.float64)[: ksteps * p * p].reshape(ksteps, p, p)
        bb = np.frombuffer(be, dtype=np.float64)[: ksteps * p * p].reshape(ksteps, p, p)
        return {"X": Xt.t().cpu(), "R": R.t().cpu(), "D": D.t().cpu(),
                "alphas": a.transpose(0, 2, 1).copy(), "betas": bb.transpose(0, 2, 1).copy()}

    def convert_matrix(self, A: torch.Tensor, prec: str):
        """The low-precision copy of A streamed by a ``prec`` solve: a float32 n x n
        tensor (fp32), or the (hi, lo) BF16 planes as int16 bit patterns (bf16x2).
        The result keeps A's element order when A is row-major contiguous (the
        library reads such a tensor as the column-major matrix A^T)."""
        aptr, lda, keep = _colmajor_matrix(A)
        n = A.shape[0]
        if prec == "fp32":
            hi = torch.empty(n, n, dtype=torch.float32, device=A.device)
            lo = None
        else:
            hi = torch.empty(n, n, dtype=torch.int16, device=A.device)
            lo = torch.empty(n, n, dtype=torch.int16, device=A.device)
        torch.cuda.synchronize(A.device)
        st = self.lib.ccg_convert_matrix(self.h, n, aptr, lda, PREC[prec], hi.data_ptr(),
                                         None if lo is None else lo.data_ptr())
        if st < 0:
            raise self._err(st)
        del keep
        return hi if lo is None else (hi, lo)

    def tune_ad(self, prec: str, p: int, n: int, cw: int, reps: int = 10, nw: int = 4,
                batched: bool = False) -> float:
        """Microseconds per A.D launch with tile shape (cw, nw), of the single-system
        or (batched) the batched kernel (see ccg_tune_ad)."""
        us = ctypes.c_double()
        st = self.lib.ccg_tune_ad(self.h, PREC[prec], p, n, cw, nw, int(batched), reps, ctypes.byref(us))
        if st != 0:
            raise self._err(st)
        return us.value

    def stream_probe(self, n: int, cols: int, dcols: int = 0, stagger=True, reps: int = 20,
                     waves: int = 4) -> float:
        """Median microseconds of the read-only stream of an n x n FP64 matrix, cols
        columns per workgroup of waves x 64 threads, plus an n x dcols block per
        workgroup (ccg_stream_probe); stagger=2: the grid-stride read of the same
        bytes by n / cols workgroups."""
        us = ctypes.c_double()
        st = self.lib.ccg_stream_probe(self.h, n, cols, dcols, int(stagger), waves, reps, ctypes.byref(us))
        if st != 0:
            raise self._err(st)
        return us.value

    def kernel_time(self, reset: bool = False, with_bytes: bool = False):
        """(ms, launches) of the timed A.D passes, and their algorithmic bytes with
        with_bytes (ccg_kernel_time)."""
        ms = ctypes.c_double()
        cnt = ctypes.c_longlong()
        nbytes = ctypes.c_double()
        self.lib.ccg_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(nbytes), int(reset))
        if with_bytes:
            return ms.value, cnt.value, nbytes.value
        return ms.value, cnt.value
