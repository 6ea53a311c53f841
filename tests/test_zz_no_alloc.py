"""accsk_solve_dense_noalloc (the entry point that allocates no device memory)
against accsk_solve_dense, through the C ABI.

Both entry points run the same routing and kernels with every reduction in a
fixed order, so on the same inputs they must return bitwise identical
potentials, iteration counts, errors and values; only the workspace differs
(one fixed per-device array instead of stream-ordered allocations).  Each
result is also held to the parity bar of the dense tests: FP64 two-sided
marginal error at the returned potentials <= tol on the oracle.

Three calls in a row on the shared array, each smaller than the one before
(a cooperative launch of workgroup-wide rows, a cooperative launch of
wave-owned rows, one workgroup), then the first shape again: what an earlier
call left in the array must not leak into a later one.
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [  # n, m, eps, seed: routes of decreasing size
    (2048, 3000, 3e-3, 31),   # cooperative, rows spread over the workgroup (m > 2048)
    (700, 500, 1e-2, 32),     # cooperative, wave-owned rows (m <= 1024)
    (200, 150, 1e-2, 33),     # one workgroup (n*m <= 65536)
    (2048, 3000, 3e-3, 31),   # the first shape again, after smaller calls
]


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def test_noalloc_matches_solve_dense(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    tol = 1e-6
    for n, m, eps, seed in CASES:
        print("case noalloc", n, m, eps, seed, flush=True)
        p = W.random_dense(seed, n, m, eps=eps, a_kind="dirichlet")
        C = _dev(torch, p["C32"], torch.float32)
        a = _dev(torch, p["a"], torch.float64)
        b = _dev(torch, p["b"], torch.float64)
        f1, g1, r1 = accsk.solve_dense(C, a, b, eps, tol=tol)
        f2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        g2 = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
        _, _, r2 = accsk.solve_dense_noalloc(C, a, b, eps, tol=tol, f_out=f2, g_out=g2)
        torch.cuda.synchronize()
        print("  It", r1["iters"], r2["iters"], "err", r1["marginal_err"], r2["marginal_err"],
              "ms", r1["kernel_ms"], r2["kernel_ms"], flush=True)
        assert r2["status"] == accsk.OK and r2["converged"] == 1
        for k in ("iters", "sinkhorn_steps", "fallback_steps", "fval_increases", "marginal_err", "eot_value",
                  "transport_cost", "dual_fval", "converged", "status"):
            assert r1[k] == r2[k], (k, r1[k], r2[k])
        assert torch.equal(f1, f2) and torch.equal(g1, g2)
        assert r2["kernel_ms"] > 0.0  # device clock of the solve
        fh, gh = f2.cpu().numpy(), g2.cpu().numpy()
        an, bn = p["a"] / p["a"].sum(), p["b"] / p["b"].sum()
        ev = O.evaluate(p["C32"].astype(np.float64), eps, an, bn, fh, gh)
        assert ev["err"] <= tol, ev


def test_noalloc_limits(torch_gpu):
    """Sizes beyond the fixed array, and m > 8192, are refused before any work is enqueued."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    L = accsk.lib()
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")  # never read: every call fails its checks
    ptr = ctypes.c_void_p(buf.data_ptr())
    prm = accsk.default_params(eps=1e-2)
    r = accsk.Result()
    # n = 200000 rows of 8192 columns needs more workspace than the array holds
    assert L.accsk_solve_dense_noalloc(ptr, 200000, 8192, 8192, ptr, ptr, ctypes.byref(prm), ptr, ptr,
                                       ctypes.byref(r), None) == accsk.SHAPE
    assert L.accsk_solve_dense_noalloc(ptr, 4, 9000, 9000, ptr, ptr, ctypes.byref(prm), ptr, ptr,
                                       ctypes.byref(r), None) == accsk.SHAPE
    torch.cuda.synchronize()
