"""Stability monitor and the optional restart safeguard, on all three GPU solvers.

The reduced dual objective f(x) = 1 - <u,a> - <x,b> (Lemma coercivity) falls
along plain Sinkhorn (Lemma sinkhorn-descent); Acc-Sinkhorn with the hand-off
of w printed in Algorithm A2MD-homotopy (LITERAL) oscillates and raises it
thousands of times at small eps.  The library counts rises above 1e-8 + 1e-12|f|
(fval_increases); with ACCSK_FLAG_RESTART it resets w <- alpha x at each rise.
The oracle implements the same rule.  Counts are compared loosely (a rise close
to the threshold may be seen by one side only); solutions are compared at tol.
"""
import numpy as np
import pytest

from oracle import oracle as O

from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _oracle(C, a, b, eps, rule, restart, method=O.ACC):
    return O.solve(C, a, b, eps, tol=1e-6 * 15 / 16, method=method, mu0=0.25, m0=5, w_rule=rule,
                   restart=restart, max_iter=50000)


def _check(r, f, g, C, an, bn, eps, o):
    ev = O.evaluate(C, eps, an, bn, f, g)
    assert r["converged"] == 1 and ev["err"] <= 1e-6 * 1.0001
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * eps + 1e-12 * abs(ev["dual"])
    eo = O.evaluate(C, eps, an, bn, o["f"], o["g"])
    assert abs(ev["dual"] - eo["dual"]) <= 1e-6 * eps * 10 + 1e-9 * abs(eo["dual"])


@pytest.mark.parametrize("path", ["dense", "batch", "tiled"])
def test_monitor_and_restart(torch_gpu, path):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    # 256 x 256 runs on one workgroup; the cooperative dense solver takes 300 x 300
    side = 300 if path == "dense" else 256
    p = W.small_uniform(seed=1, n=side, m=side)
    eps = 1e-3
    C = p["C32"].astype(np.float64)
    an, bn = p["a"], p["b"]
    X = np.asarray(p["X"], np.float32)
    Y = np.asarray(p["Y"], np.float32)
    if path == "tiled":  # the same points, cost formed on the fly (exact FP64 cost, max-normalized)
        raw = O.cost_points(0, X, Y, 1.0)
        s = float(raw.max())
        C = raw / s
    o_plain = _oracle(C, an, bn, eps, O.W_LITERAL, False)
    o_rst = _oracle(C, an, bn, eps, O.W_LITERAL, True)
    o_sk = _oracle(C, an, bn, eps, O.W_LITERAL, False, method=O.SINKHORN)
    out = {}
    for name, meth, flags in (("plain", accsk.ACC, 0), ("restart", accsk.ACC, accsk.FLAG_RESTART),
                              ("sinkhorn", accsk.SINKHORN, 0)):
        kw = dict(method=meth, w_rule=accsk.W_LITERAL, flags=flags, max_iter=50000)
        if path == "dense":
            f, g, r = accsk.solve_dense(_dev(torch, p["C32"], torch.float32), _dev(torch, an, torch.float64),
                                        _dev(torch, bn, torch.float64), eps, **kw)
        elif path == "batch":
            outs, res, _ = accsk.solve_batch([(_dev(torch, p["C32"], torch.float32), _dev(torch, an, torch.float64),
                                               _dev(torch, bn, torch.float64), eps)], **kw)
            (f, g), r = outs[0], res[0]
        else:
            f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                           _dev(torch, an, torch.float64), _dev(torch, bn, torch.float64), eps,
                                           cost_scale=s, on_the_fly=True, **kw)
            r = res[0]
        torch.cuda.synchronize()
        out[name] = (f.cpu().numpy(), g.cpu().numpy(), r)
    fp, gp, rp = out["plain"]
    fr, gr, rr = out["restart"]
    fs, gs, rs = out["sinkhorn"]
    print(path, "plain It", rp["iters"], "incr", rp["fval_increases"], "(oracle", o_plain["iters"],
          o_plain["fval_increases"], ") restart It", rr["iters"], "restarts", rr["restarts"], "(oracle",
          o_rst["iters"], o_rst["restarts"], ") sinkhorn incr", rs["fval_increases"], flush=True)
    _check(rp, fp, gp, C, an, bn, eps, o_plain)
    _check(rr, fr, gr, C, an, bn, eps, o_rst)
    _check(rs, fs, gs, C, an, bn, eps, o_sk)
    # the monitor sees the LITERAL oscillation as the oracle does
    assert rp["fval_increases"] >= 0.5 * o_plain["fval_increases"] > 0
    assert rp["restarts"] == 0 and rs["restarts"] == 0
    # the safeguard removes most of the iterations, as on the oracle
    assert rr["restarts"] > 0 and rr["iters"] <= 0.5 * rp["iters"]
    assert rr["iters"] <= 2 * o_rst["iters"] + 50
    # plain Sinkhorn descends (within the threshold)
    assert rs["fval_increases"] <= 2
