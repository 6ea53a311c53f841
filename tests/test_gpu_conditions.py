"""Boundedness monitor (ACCSK_FLAG_CONDITIONS: the two conditions of Theorem
thm:condition-boundedness with the metric of eq:D, and the shifted Lyapunov
function of its proof) on the three GPU solvers, against the oracle.

The monitor runs in separate (diagnostic) kernel instantiations; it must not
change the iterates, so the potentials and iteration counts are compared
bitwise with a solve without it.  The GPU forms its column sums from FP32
exponentials (relative noise ~1e-7), so a comparison that sits at its
threshold can go either way: counts are compared with a small slack.
"""
import numpy as np
import pytest

from oracle import oracle as O

from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("w_rule", [0, 1])
@pytest.mark.parametrize("path", ["dense", "batch", "tiled"])
def test_conditions_against_oracle(torch_gpu, path, w_rule):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    side = 300 if path == "dense" else 256  # 256 x 256 runs on one workgroup
    p = W.small_uniform(seed=1, n=side, m=side)
    eps = 3e-3
    an, bn = p["a"], p["b"]
    C = p["C32"].astype(np.float64)
    X = np.asarray(p["X"], np.float32)
    Y = np.asarray(p["Y"], np.float32)
    if path == "tiled":
        raw = O.cost_points(0, X, Y, 1.0)
        s = float(raw.max())
        C = raw / s
    o = O.solve(C, an, bn, eps, tol=1e-6 * 15 / 16, mu0=0.25, m0=5, w_rule=w_rule, max_iter=20000,
                conditions=True)
    out = {}
    for flags in (0, accsk.FLAG_CONDITIONS):
        kw = dict(w_rule=w_rule, flags=flags, max_iter=20000)
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
        out[flags] = (f.cpu().numpy(), g.cpu().numpy(), r)
    f0, g0, r0 = out[0]
    f1, g1, r1 = out[accsk.FLAG_CONDITIONS]
    got = [r1["cond1_violations"], r1["cond2_violations"], r1["lyap_increases"]]
    print(path, "w_rule", w_rule, "It", r1["iters"], "(oracle", o["iters"], ") gpu counts", got, "oracle",
          o["cond_counts"], flush=True)
    assert [r0["cond1_violations"], r0["cond2_violations"], r0["lyap_increases"]] == [-1, -1, -1]
    assert r0["iters"] == r1["iters"] and np.array_equal(f0, f1) and np.array_equal(g0, g1)
    assert r1["converged"] == 1
    assert abs(r1["iters"] - o["iters"]) <= 2
    # counts: the iteration counts may differ by one or two, and a comparison at its threshold by one
    slack = 2 + abs(r1["iters"] - o["iters"])
    for k in range(3):
        assert abs(got[k] - o["cond_counts"][k]) <= slack, (k, got, o["cond_counts"])
    assert got[0] >= 5  # the first stages (alpha = 0.71, 0.5) violate condition 1


def test_conditions_refused_for_batches_and_servers(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.small_uniform(seed=2, n=64, m=64)
    prob = (_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
            _dev(torch, p["b"], torch.float64), p["eps"])
    _, _, st = accsk.solve_batch([prob, prob], flags=accsk.FLAG_CONDITIONS, raise_on_error=False)
    assert st == accsk.INVALID_ARG
    with pytest.raises(accsk.AccskError):
        accsk.Server(1 << 24, flags=accsk.FLAG_CONDITIONS)
