"""The per-step error trace of every solver route against the oracle's, entry by entry.

For each route that a single problem can take (one workgroup; cooperating
workgroups with wave-owned rows; cooperating workgroups with workgroup-wide
rows, m <= 2048 and m <= 4096; the tiled solver on an explicit cost; the tiled
solver on the fly), err_trace[k] -- the L1 marginal error (eq:l1tol) of the
iterate evaluated by Sinkhorn step k -- is compared with the FP64 oracle's error
trace for the same number of steps: |gpu - oracle| <= 2e-7 + 1e-5 |oracle| at
every k.  2e-7 is the noise of an error computed from FP32 exponentials summed
in FP64 (tests/_stopcheck.py); the relative term covers the early steps, where
the error is of order one and the two trajectories differ by FP32 rounding.
"""
import numpy as np
import pytest

from oracle import oracle as O

from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _compare(gpu_trace, r, C64, a, b, eps, method):
    from paper_2605_30267_amd import accsk
    dp = accsk.default_params()
    it = r["iters"]
    assert len(gpu_trace) == r["sinkhorn_steps"] == it + 1
    assert np.all(np.isfinite(gpu_trace))
    o = O.solve(C64, a, b, eps, tol=1e-300, max_iter=it, method=O.ACC if method == accsk.ACC else O.SINKHORN,
                mu0=dp.mu0, m0=dp.m0, w_rule=dp.w_rule, trace=True)["trace_err"]
    o = np.asarray(o)
    assert len(o) == it + 1
    dev = np.abs(gpu_trace - o)
    k = int(np.argmax(dev - (2e-7 + 1e-5 * o)))
    print("  steps", it + 1, "max |diff|", dev.max(), "at", k, "gpu", gpu_trace[k], "oracle", o[k], flush=True)
    assert np.all(dev <= 2e-7 + 1e-5 * o)
    assert gpu_trace[-1] < 1e-6 * 15 / 16


@pytest.mark.parametrize("method", [1, 0])
@pytest.mark.parametrize("n,m,eps", [(64, 80, 1e-2), (300, 260, 3e-3), (150, 2000, 1e-2), (200, 3000, 1e-2),
                                     (100, 9001, 2e-2)])
def test_trace_dense_routes(torch_gpu, n, m, eps, method):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(700 + n, n, m, eps=eps, a_kind="dirichlet")
    print("case trace", n, m, eps, "method", method, flush=True)
    f, g, r = accsk.solve_dense(_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
                                _dev(torch, p["b"], torch.float64), eps, method=method, max_iter=20000, trace=True)
    torch.cuda.synchronize()
    assert r["converged"] == 1
    _compare(r["trace"], r, p["C32"].astype(np.float64), p["a"], p["b"], eps, method)


@pytest.mark.parametrize("method", [1, 0])
def test_trace_on_the_fly(torch_gpu, method):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    rng = np.random.default_rng(77)
    X = rng.uniform(0, 1, (500, 3)).astype(np.float32)
    Y = rng.uniform(0, 1, (700, 3)).astype(np.float32)
    a, b = rng.uniform(0.5, 1.5, 500), rng.uniform(0.5, 1.5, 700)
    raw = O.cost_points(0, X, Y, 1.0)
    s = float(raw.max())
    print("case trace on the fly, method", method, flush=True)
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), 1e-2, cost_scale=s,
                                   on_the_fly=True, method=method, max_iter=20000, trace=True)
    torch.cuda.synchronize()
    r = res[0]
    assert r["converged"] == 1
    _compare(r["trace"], r, raw / s, a / a.sum(), b / b.sum(), 1e-2, method)


def test_trace_shorter_than_solve(torch_gpu):
    """A trace buffer shorter than the solve keeps its first entries and nothing else is written."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(790, 300, 260, eps=3e-3)
    C, a, b = _dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    _, _, full = accsk.solve_dense(C, a, b, 3e-3, trace=True)
    buf = torch.full((12,), -1.0, dtype=torch.float64, device="cuda")
    prm = accsk.default_params(eps=3e-3, err_trace=buf.data_ptr(), trace_len=10)
    f = torch.empty(300, dtype=torch.float64, device="cuda")
    g = torch.empty(260, dtype=torch.float64, device="cuda")
    import ctypes
    r = accsk.Result()
    st = accsk.lib().accsk_solve_dense(accsk._ptr(C), 300, 260, 260, accsk._ptr(a), accsk._ptr(b), ctypes.byref(prm),
                                       accsk._ptr(f), accsk._ptr(g), ctypes.byref(r), accsk._stream_ptr())
    torch.cuda.synchronize()
    assert st == accsk.OK and r.sinkhorn_steps > 12
    got = buf.cpu().numpy()
    assert np.array_equal(got[:10], full["trace"][:10]) and np.all(got[10:] == -1.0)
