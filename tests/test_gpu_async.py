"""Stream-ordered entry points (accsk_solve_dense_async, accsk_solve_batch_strided_async,
accsk_solve_points_batched_async) against their blocking forms, through the C ABI.

The two forms run the same routing and kernels with fixed-order reductions, so
the potentials, iteration counts, errors and values must be bitwise identical;
only where the result record lives differs (device memory, written by the
device).  Several solves are enqueued back to back with no host wait between
them and checked after a single synchronization; the stream must still be busy
when the enqueueing calls return (the calls do not wait for the solve).
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("iters", "sinkhorn_steps", "fallback_steps", "fval_increases", "restarts", "marginal_err", "eot_value",
          "transport_cost", "dual_fval", "converged", "status")


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _same(r_host, r_dev, name):
    for k in FIELDS:
        assert r_host[k] == r_dev[k], (name, k, r_host[k], r_dev[k])
    assert r_dev["kernel_ms"] > 0.0, name


def test_dense_async_back_to_back(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    probs = [W.gmm_dense(seed=2, n=4096, m=4096, eps=1e-3),          # cooperative, several ms
             W.random_dense(41, 2048, 3000, eps=3e-3, a_kind="dirichlet"),
             W.random_dense(42, 200, 150, eps=1e-2)]                  # one workgroup (FP64 re-evaluation)
    dev = []
    for p in probs:
        dev.append((_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
                    _dev(torch, p["b"], torch.float64), p["eps"]))
    torch.cuda.synchronize()
    print("case dense async x3", flush=True)
    outs = [accsk.solve_dense_async(C, a, b, eps) for C, a, b, eps in dev]
    busy = not torch.cuda.current_stream().query()  # the first solve takes milliseconds
    torch.cuda.synchronize()
    assert busy, "the stream-ordered calls waited for their work"
    for k, ((C, a, b, eps), (f, g, rec), p) in enumerate(zip(dev, outs, probs)):
        rd = accsk.read_records(rec)[0]
        fh, gh, rh = accsk.solve_dense(C, a, b, eps)
        torch.cuda.synchronize()
        print("  problem", k, "It", rd["iters"], rh["iters"], "err", rd["marginal_err"], flush=True)
        _same(rh, rd, "dense %d" % k)
        assert torch.equal(f, fh) and torch.equal(g, gh)
        if k > 0:  # FP64 check on the oracle (the 4096^2 one is covered by the dense tests)
            an, bn = p["a"] / p["a"].sum(), p["b"] / p["b"].sum()
            ev = O.evaluate(p["C32"].astype(np.float64), eps, an, bn, f.cpu().numpy(), g.cpu().numpy())
            assert ev["err"] <= 1e-6, ev


def test_dense_async_outcomes_in_record(torch_gpu):
    """Outcomes found on the device go to the record; the call itself returns OK."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(43, 300, 260, eps=1e-2)
    C = _dev(torch, p["C32"], torch.float32)
    a = _dev(torch, p["a"], torch.float64)
    b = _dev(torch, p["b"], torch.float64)
    bad = a.clone()
    bad[7] = -1.0
    print("case async outcomes", flush=True)
    _, _, r1 = accsk.solve_dense_async(C, a, b, p["eps"], max_iter=3)
    _, _, r2 = accsk.solve_dense_async(C, bad, b, p["eps"])
    d1, d2 = accsk.read_records(r1)[0], accsk.read_records(r2)[0]
    assert d1["status"] == accsk.NOT_CONVERGED and d1["converged"] == 0 and d1["iters"] == 3
    assert d2["status"] == accsk.INVALID_ARG
    L = accsk.lib()
    prm = accsk.default_params(eps=1e-2)
    assert L.accsk_solve_dense_async(accsk._ptr(C), 300, 260, 260, accsk._ptr(a), accsk._ptr(b), ctypes.byref(prm),
                                     accsk._ptr(a), accsk._ptr(b), None, None) == accsk.INVALID_ARG


def test_batch_strided_async(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    B, n, m = 12, 256, 256
    ps = [W.small_uniform(seed=100 + k, n=n, m=m) for k in range(B)]
    C = _dev(torch, np.stack([q["C32"] for q in ps]), torch.float32)
    a = _dev(torch, np.stack([q["a"] for q in ps]), torch.float64)
    b = _dev(torch, np.stack([q["b"] for q in ps]), torch.float64)
    eps = ps[0]["eps"]
    print("case strided async", B, n, m, flush=True)
    f1, g1, rec = accsk.solve_batch_strided_async(C, a, b, eps)
    f2, g2, res, st = accsk.solve_batch_strided(C, a, b, eps)
    recs = accsk.read_records(rec)
    assert st == accsk.OK and len(recs) == B
    for k in range(B):
        for fld in FIELDS:
            assert res[fld][k] == recs[k][fld], (k, fld)
    assert torch.equal(f1, f2) and torch.equal(g1, g2)


@pytest.mark.parametrize("on_the_fly", [False, True])
def test_points_async(torch_gpu, on_the_fly):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    rng = np.random.default_rng(44)
    B, n, m, d = 3, 300, 500, 3
    X = _dev(torch, rng.uniform(0, 1, (B, n, d)), torch.float32)
    Y = _dev(torch, rng.uniform(0, 1, (B, m, d)), torch.float32)
    a = _dev(torch, np.full((B, n), 1.0 / n), torch.float64)
    b = _dev(torch, np.full((B, m), 1.0 / m), torch.float64)
    print("case points async on_the_fly", on_the_fly, flush=True)
    f1, g1, rec = accsk.solve_points_async(X, Y, a, b, 1e-2, cost_scale=3.0, on_the_fly=on_the_fly)
    f2, g2, res = accsk.solve_points(X, Y, a, b, 1e-2, cost_scale=3.0, on_the_fly=on_the_fly)
    recs = accsk.read_records(rec)
    for k in range(B):
        _same(res[k], recs[k], "points %d" % k)
    assert torch.equal(f1, f2) and torch.equal(g1, g2)
