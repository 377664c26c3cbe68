"""Where a run of the oracle restarts (shared by the oracle pins and the GPU tests).

The stop rule (Alg. 4's smallest-agent test on the recurrence residual, confirmed by
the explicit residual) restarts the agents from R = D = B - A X when the explicit
residual fails the test.  A run capped at maxit = k reports that restart exactly
when it happens at the top of step k or earlier, so the first restart step is the
smallest such k (the restart count is monotone in maxit).
"""
import oracle


def first_restart_step(A, b, X0, tol, hi, lib=None):
    """Smallest k <= hi such that the oracle run with maxit = k has restarted, or
    None if the run with maxit = hi has not."""
    def restarted(k):
        return oracle.ccg(A, b, X0, tol=tol, maxit=k, lib=lib)["restarts"] >= 1

    if not restarted(hi):
        return None
    lo = 0                      # the explicit and recurrence residuals coincide at k = 0
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if restarted(mid):
            hi = mid
        else:
            lo = mid
    return hi
