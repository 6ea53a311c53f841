"""GPU tests of the serving loop (persistent kernel, continuous batching).

* Every served request matches the FP64 oracle run on the oracle's own cost
  (rounded to FP32 as the server stores it): FP64 marginal error <= tol, EOT
  value, stopping iterate (tests/_stopcheck.py).
* A request gives the same bits alone and mixed with other requests, with a
  small HBM budget (requests wait for arena space) and a large one.
* For m <= 128 the server runs the same solver configuration as the batched
  point-cloud solve, so the two give the same bits.
* Errors, and a relaunch after the persistent kernel has gone idle.
"""
import time

import numpy as np
import pytest

from oracle import oracle as O

from _stopcheck import check_stop
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _reqs(seed, count, nmin=8, nmax=256, d=300):
    return W.word_requests(seed=seed, count=count, d=d, nmin=nmin, nmax=nmax)


def _submit(torch, srv, r, kind=1, scale=1.0):
    return srv.submit(_dev(torch, r["X"], torch.float32), _dev(torch, r["Y"], torch.float32),
                      _dev(torch, r["a"], torch.float64), _dev(torch, r["b"], torch.float64), r["eps"], kind=kind,
                      cost_scale=scale)


def _run_all(torch, srv, reqs, kind=1, scale=1.0):
    tickets = [_submit(torch, srv, r, kind, scale) for r in reqs]
    torch.cuda.synchronize()
    outs = [srv.wait(t, timeout=120.0) for t in tickets]
    return [(f.cpu().numpy(), g.cpu().numpy(), res) for f, g, res, _ in outs]


def test_serve_matches_oracle(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    reqs = _reqs(seed=21, count=12)
    dp = accsk.default_params()
    with accsk.Server(hbm_budget=64 << 20) as srv:
        outs = _run_all(torch, srv, reqs)
    for k, (r, (f, g, res)) in enumerate(zip(reqs, outs)):
        C32 = O.cost_points(1, r["X"], r["Y"], 1.0).astype(np.float32).astype(np.float64)
        an, bn = r["a"] / r["a"].sum(), r["b"] / r["b"].sum()
        ev = O.evaluate(C32, r["eps"], an, bn, f, g)
        print("req", k, C32.shape, r["eps"], "It", res["iters"], "err", ev["err"], "device ms", res["kernel_ms"],
              flush=True)
        assert res["status"] == 0 and res["converged"] == 1, res
        assert ev["err"] <= 1e-6 * 1.001
        assert abs(res["eot_value"] - ev["dual"]) <= 2e-7 * r["eps"] + 1e-12 * abs(ev["dual"])
        check_stop(C32, an, bn, r["eps"], 1e-6, O.ACC, res["iters"], dp.mu0, dp.m0, dp.w_rule)


@pytest.mark.parametrize("budget", [2 << 20, 256 << 20])
def test_serve_alone_vs_mixed(torch_gpu, budget):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    probes = _reqs(seed=22, count=3)
    others = _reqs(seed=23, count=60)
    with accsk.Server(hbm_budget=budget) as srv:
        alone = [_run_all(torch, srv, [r])[0] for r in probes]
        mix = others[:20] + [probes[0]] + others[20:40] + [probes[1]] + others[40:] + [probes[2]]
        tickets = [_submit(torch, srv, r) for r in mix]
        torch.cuda.synchronize()
        seen_wait = False
        for _ in range(20):
            seen_wait |= srv.info()["waiting"] > 0
        outs = [srv.wait(t, timeout=120.0) for t in tickets]
        info = srv.info()
    pos = [20, 41, 62]
    for k, p in enumerate(pos):
        f, g, res, _ = outs[p]
        fa, ga, ra = alone[k]
        assert res["iters"] == ra["iters"] and res["converged"] == 1
        assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(g.cpu().numpy(), ga)
        assert res["eot_value"] == ra["eot_value"]
    assert all(o[2]["converged"] == 1 for o in outs)
    assert info["in_flight"] == 0 and info["waiting"] == 0
    print("budget", budget, "saw waiting requests:", seen_wait, info, flush=True)


def test_serve_admission_binds(torch_gpu):
    """Admission by HBM footprint: an arena that holds one 256 x 256 cost
    (256 KiB) plus one 96 x 160 cost (60 KiB), and five requests submitted at
    once: big A, big B, small c, big D, small e (B and D sized like A).
    A is admitted at once; B waits for A's block (its first-fit search fails),
    the small c goes first into the remaining space; B is admitted only after A
    completed and D only after B.  Each result is bitwise the one the request
    gives alone, and the server's admission counters record the waits."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    rng = np.random.default_rng(26)

    def req(n, m, eps):
        X = W.unit_rows(rng, n, 300).astype(np.float32)
        Y = W.unit_rows(rng, m, 300).astype(np.float32)
        return dict(X=X, Y=Y, a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), eps=eps)

    big = [req(256, 256, 1e-3), req(256, 256, 3e-3), req(256, 256, 1e-3)]
    small = [req(96, 160, 1e-2), req(96, 160, 3e-3)]
    order = [big[0], big[1], small[0], big[2], small[1]]
    budget = 256 * 256 * 4 + 96 * 160 * 4
    with accsk.Server(hbm_budget=budget) as srv:
        alone = [_run_all(torch, srv, [r])[0] for r in order]
        st0 = srv.admission()
        assert st0["space_waited"] == 0
        tickets = [_submit(torch, srv, r) for r in order]
        torch.cuda.synchronize()
        outs = [srv.wait(t, timeout=120.0) for t in tickets]
        st = srv.admission()
    tA, tB, tc, tD, te = [o[3] for o in outs]  # (submit, admit, done) on the host clock
    print("admission", st, flush=True)
    print("  A admit %.6f done %.6f | B admit %.6f done %.6f | c admit %.6f | D admit %.6f"
          % (tA[1], tA[2], tB[1], tB[2], tc[1], tD[1]), flush=True)
    assert tB[1] >= tA[2] and tD[1] >= tB[2]  # each big one admitted after the previous big one completed
    assert tc[1] < tB[1]  # the small request went ahead of the waiting big one
    assert st["space_waited"] >= 2 and st["fit_failures"] >= 2 and st["overtakes"] >= 1
    assert st["peak_bytes_in_use"] <= budget
    for (f, g, res, _), (fa, ga, ra) in zip(outs, alone):
        assert res["converged"] == 1 and res["iters"] == ra["iters"]
        assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(g.cpu().numpy(), ga)


@pytest.mark.parametrize("split", [0, 3])
def test_serve_equals_batched_points(torch_gpu, split):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    reqs = _reqs(seed=24, count=6, nmin=8, nmax=128)
    with accsk.Server(hbm_budget=64 << 20, split=split) as srv:
        outs = _run_all(torch, srv, reqs)
    for r, (f, g, res) in zip(reqs, outs):
        fb, gb, rb = accsk.solve_points(_dev(torch, r["X"], torch.float32), _dev(torch, r["Y"], torch.float32),
                                        _dev(torch, r["a"], torch.float64), _dev(torch, r["b"], torch.float64),
                                        r["eps"], kind=accsk.COSINE, split=split)
        torch.cuda.synchronize()
        assert rb[0]["iters"] == res["iters"]
        assert np.array_equal(fb.cpu().numpy(), f) and np.array_equal(gb.cpu().numpy(), g)


def test_serve_large_columns_and_sqeuclid(torch_gpu):
    """m in (128, 512]: other solver configurations; squared Euclidean costs."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    rng = np.random.default_rng(25)
    reqs = []
    for n, m, d in [(300, 200, 3), (512, 512, 16), (77, 400, 64), (5, 300, 2)]:
        X = rng.uniform(0, 1, (n, d)).astype(np.float32)
        Y = rng.uniform(0, 1, (m, d)).astype(np.float32)
        reqs.append(dict(X=X, Y=Y, a=rng.uniform(0.5, 1.5, n), b=rng.uniform(0.5, 1.5, m), eps=1e-2, d=d))
    dp = accsk.default_params()
    with accsk.Server(hbm_budget=64 << 20, method=accsk.ACC) as srv:
        outs = _run_all(torch, srv, reqs, kind=0, scale=2.0)
    for r, (f, g, res) in zip(reqs, outs):
        C32 = O.cost_points(0, r["X"], r["Y"], 2.0).astype(np.float32).astype(np.float64)
        an, bn = r["a"] / r["a"].sum(), r["b"] / r["b"].sum()
        ev = O.evaluate(C32, r["eps"], an, bn, f, g)
        assert res["converged"] == 1 and ev["err"] <= 1e-6 * 1.001
        check_stop(C32, an, bn, r["eps"], 1e-6, O.ACC, res["iters"], dp.mu0, dp.m0, dp.w_rule)


def test_serve_sinkhorn(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    reqs = _reqs(seed=26, count=4, nmax=96)
    with accsk.Server(hbm_budget=16 << 20, method=accsk.SINKHORN) as srv:
        outs = _run_all(torch, srv, reqs)
    for r, (f, g, res) in zip(reqs, outs):
        C32 = O.cost_points(1, r["X"], r["Y"], 1.0).astype(np.float32).astype(np.float64)
        an, bn = r["a"] / r["a"].sum(), r["b"] / r["b"].sum()
        ev = O.evaluate(C32, r["eps"], an, bn, f, g)
        assert res["converged"] == 1 and ev["err"] <= 1e-6 * 1.001
        check_stop(C32, an, bn, r["eps"], 1e-6, O.SINKHORN, res["iters"], 0.25, 5, 1)


def test_serve_errors_and_relaunch(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    r = _reqs(seed=27, count=1, nmin=40, nmax=40)[0]
    big = dict(r, X=np.zeros((513, 300), np.float32), a=np.ones(513))
    with accsk.Server(hbm_budget=4096) as srv:
        with pytest.raises(accsk.AccskError) as e:
            _submit(torch, srv, big)
        assert e.value.status == accsk.SHAPE
        with pytest.raises(accsk.AccskError) as e:
            _submit(torch, srv, r)  # 40 x 40 x 4 bytes > 4096-byte arena
        assert e.value.status == accsk.OOM
        with pytest.raises(accsk.AccskError) as e:
            srv.poll(12345)
        assert e.value.status == accsk.INVALID_ARG
    with accsk.Server(hbm_budget=1 << 20) as srv:
        f1, g1, r1 = _run_all(torch, srv, [r])[0]
        n1 = srv.info()["launches"]
        time.sleep(0.6)  # the persistent kernel ends after 0.25 s without requests
        f2, g2, r2 = _run_all(torch, srv, [r])[0]
        n2 = srv.info()["launches"]
    assert n2 == n1 + 1
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2) and r1["iters"] == r2["iters"]
