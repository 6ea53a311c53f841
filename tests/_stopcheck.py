"""Stopping-iteration check shared by the GPU parity tests.

The library stops at the first iterate whose self-computed L1 marginal error
(eq:l1tol) is below thr = tol*(1 - 1/16).  Its error estimate comes from FP32
exponentials summed in FP64 and carries an absolute noise of order
1e-7 * sum(b) = 1e-7.  So, with the oracle's FP64 error trace err_o[k] of the
same iteration, the GPU's stopping iterate k_g must satisfy
    err_o[k_g] <= thr + DELTA     and     err_o[k] >= thr - DELTA for k < k_g,
with DELTA = 1.5e-7: it did not stop early and did not skip a clearly
converged iterate.  This holds for the non-monotone error sequence of
Acc-Sinkhorn, where a fixed +-N window on k does not.
"""
import numpy as np

from oracle import oracle as O

STOP = 1.0 - 1.0 / 16.0
DELTA = 1.5e-7


def check_stop(C64, a, b, eps, tol, method, it_gpu, mu0, m0, w_rule):
    thr = tol * STOP
    tr = O.solve(C64, a, b, eps, tol=1e-300, max_iter=it_gpu, method=method, mu0=mu0, m0=m0,
                 w_rule=w_rule, trace=True)["trace_err"]
    assert len(tr) == it_gpu + 1
    assert tr[it_gpu] <= thr + DELTA, (it_gpu, tr[it_gpu], thr)
    if it_gpu > 0:
        assert np.min(tr[:it_gpu]) >= thr - DELTA, (np.argmin(tr[:it_gpu]), np.min(tr[:it_gpu]), thr)
