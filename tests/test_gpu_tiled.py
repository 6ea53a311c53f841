"""GPU parity of the tiled solver: costs formed on the fly from point clouds
(never stored) and explicit costs with m > 8192.

On the fly the exponent arguments are formed in FP64 from the FP32 points, so
the solve is judged against the FP64 oracle on the exact FP64 cost: FP64
marginal error <= tol (plus the FP64 rounding of the argument, far below it),
EOT value within eps * 2e-7 (FP32 exponentials in the mass), <C,P> to 1e-6
relative, and the stopping iterate against the oracle's error trace.
At the full colour-transfer size (n = m = 32768, d = 3, eps = 1e-3) the
oracle checks sampled rows and columns of the plan one by one.
"""
import numpy as np
import pytest

from oracle import oracle as O

from _stopcheck import check_stop
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _points(seed, n, m, d, kind):
    rng = np.random.default_rng(seed)
    if kind == 1:
        return W.unit_rows(rng, n, d).astype(np.float32), W.unit_rows(rng, m, d).astype(np.float32)
    return rng.uniform(0, 1, (n, d)).astype(np.float32), rng.uniform(0, 1, (m, d)).astype(np.float32)


# d <= 3 runs the FP64 matrix-core sweeps: cosine included, and 40000 rows give
# every wave several 16-row tiles (rounds) on 256 blocks
CASES = [(0, 500, 700, 3, 1e-2), (1, 300, 200, 8, 3e-3), (0, 64, 1500, 16, 2e-2), (0, 5, 3000, 2, 1e-2),
         (0, 1, 1, 1, 1e-1), (0, 2000, 64, 3, 1e-3), (1, 77, 9000, 4, 1e-2), (1, 300, 700, 3, 3e-3),
         (0, 40000, 40, 2, 2e-2), (1, 1000, 2600, 3, 3e-3)]


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("kind,n,m,d,eps", CASES)
def test_on_the_fly_matches_oracle(torch_gpu, kind, n, m, d, eps, method):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _points(100 + n + m, n, m, d, kind)
    rng = np.random.default_rng(n * m)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    raw = O.cost_points(kind, X, Y, 1.0)
    s = float(raw.max()) if kind == 0 else 1.0
    C = raw / s
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps, kind=kind,
                                   cost_scale=s, on_the_fly=True, method=method)
    torch.cuda.synchronize()
    r = res[0]
    an, bn = a / a.sum(), b / b.sum()
    ev = O.evaluate(C, eps, an, bn, f.cpu().numpy(), g.cpu().numpy())
    print((kind, n, m, d, eps, method), "It", r["iters"], "err", ev["err"], "fallback", r["fallback_steps"],
          "ms", r["kernel_ms"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1, r
    assert ev["err"] <= 1e-6 * 1.0001
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * eps + 1e-12 * abs(ev["dual"])
    assert abs(r["transport_cost"] - ev["cost"]) <= 1e-6 * abs(ev["cost"]) + 1e-13
    dp = accsk.default_params()
    check_stop(C, an, bn, eps, 1e-6, O.ACC if method == 1 else O.SINKHORN, r["iters"], dp.mu0, dp.m0, dp.w_rule)


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_tiled_explicit_large_m(torch_gpu, eps):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(seed=61, n=150, m=9001, eps=eps, a_kind="dirichlet")
    C = _dev(torch, p["C32"], torch.float32)
    f, g, r = accsk.solve_dense(C, _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64), eps)
    torch.cuda.synchronize()
    C64 = p["C32"].astype(np.float64)
    ev = O.evaluate(C64, eps, p["a"], p["b"], f.cpu().numpy(), g.cpu().numpy())
    print("explicit m=9001 eps", eps, "It", r["iters"], "err", ev["err"], "fallback", r["fallback_steps"], flush=True)
    assert r["converged"] == 1 and ev["err"] <= 1e-6 * 1.0001
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * eps + 1e-12 * abs(ev["dual"])
    dp = accsk.default_params()
    check_stop(C64, p["a"], p["b"], eps, 1e-6, O.ACC, r["iters"], dp.mu0, dp.m0, dp.w_rule)


@pytest.mark.parametrize("kind,n,m,d", [(0, 300, 257, 3), (1, 129, 1000, 300), (0, 17, 5, 1), (0, 2000, 1500, 3)])
def test_cost_max_points(torch_gpu, kind, n, m, d):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _points(7 + n, n, m, d, kind)
    got = accsk.cost_max_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), kind=kind)
    ref = O.cost_points(kind, X, Y, 1.0).max()
    assert abs(got - ref) <= 1e-15 * max(1.0, abs(ref))


def test_color_transfer_full_size(torch_gpu):
    """n = m = 32768 RGB points, eps = 1e-3, cost / exact max, formed on the fly.

    The FP64 oracle evaluates the returned potentials on the exact cost over all
    2^30 entries (each formed from the points when used, nothing n x m stored):
    two-sided L1 marginal error <= tol, and the dual value."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.color_points(seed=3, n=32768, m=32768, eps=1e-3)
    Xd, Yd = _dev(torch, p["X"], torch.float32), _dev(torch, p["Y"], torch.float32)
    s = accsk.cost_max_points(Xd, Yd)
    f, g, res = accsk.solve_points(Xd, Yd, _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64),
                                   p["eps"], cost_scale=s, on_the_fly=True)
    torch.cuda.synchronize()
    r = res[0]
    print("colour transfer 32768^2: It", r["iters"], "steps", r["sinkhorn_steps"], "err", r["marginal_err"],
          "kernel ms", r["kernel_ms"], "fallback", r["fallback_steps"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1
    f, g = f.cpu().numpy(), g.cpu().numpy()
    X, Y = p["X"].astype(np.float64), p["Y"].astype(np.float64)
    an, bn = p["a"] / p["a"].sum(), p["b"] / p["b"].sum()
    ev = O.evaluate_points(0, X, Y, s, p["eps"], an, bn, f, g)
    print("  FP64 on the exact cost: row err", ev["row_err"], "col err", ev["col_err"], "dual", ev["dual"],
          flush=True)
    assert ev["err"] <= 1e-6
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * p["eps"] + 1e-12 * abs(ev["dual"])
    rng = np.random.default_rng(0)
    # sampled rows: the row solve is exact, so each row marginal matches a_i to FP32-exponential accuracy
    for i in rng.choice(32768, 16, replace=False):
        Ci = ((X[i] - Y) ** 2).sum(axis=1) / s
        ri = np.exp((f[i] + g - Ci) / p["eps"]).sum()
        assert abs(ri - an[i]) <= 1e-6 * an[i] + 1e-300


def test_tiled_errors_and_limits(torch_gpu):
    """Invalid and non-finite inputs on both tiled paths, and the iteration cap."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(seed=62, n=40, m=9001, eps=1e-2)
    Cd = _dev(torch, p["C32"], torch.float32)
    a, b = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    bad = a.clone()
    bad[3] = 0.0
    assert accsk.solve_dense(Cd, bad, b, 1e-2, raise_on_error=False)[2]["status"] == accsk.INVALID_ARG
    bad[3] = float("nan")
    assert accsk.solve_dense(Cd, bad, b, 1e-2, raise_on_error=False)[2]["status"] == accsk.NONFINITE
    Cn = Cd.clone()
    Cn[5, 7] = float("nan")
    assert accsk.solve_dense(Cn, a, b, 1e-2, raise_on_error=False)[2]["status"] == accsk.NONFINITE
    r = accsk.solve_dense(Cd, a, b, 1e-2, tol=1e-300, max_iter=3, raise_on_error=False)[2]
    assert r["status"] == accsk.NOT_CONVERGED and r["iters"] == 3 and r["sinkhorn_steps"] == 4
    # on the fly: a NaN point, a zero weight, the cap
    X, Y = _points(5, 30, 50, 3, 0)
    Xd, Yd = _dev(torch, X, torch.float32), _dev(torch, Y, torch.float32)
    aa = _dev(torch, np.full(30, 1 / 30), torch.float64)
    bb = _dev(torch, np.full(50, 1 / 50), torch.float64)
    Xn = Xd.clone()
    Xn[2, 1] = float("nan")
    r = accsk.solve_points(Xn, Yd, aa, bb, 1e-2, on_the_fly=True, raise_on_error=False)[2][0]
    assert r["status"] == accsk.NONFINITE
    a0 = aa.clone()
    a0[0] = 0.0
    r = accsk.solve_points(Xd, Yd, a0, bb, 1e-2, on_the_fly=True, raise_on_error=False)[2][0]
    assert r["status"] == accsk.INVALID_ARG
    r = accsk.solve_points(Xd, Yd, aa, bb, 1e-2, on_the_fly=True, tol=1e-300, max_iter=0, raise_on_error=False)[2][0]
    assert r["status"] == accsk.NOT_CONVERGED and r["iters"] == 0 and r["sinkhorn_steps"] == 1
    with pytest.raises(accsk.AccskError) as e:  # d = 17 > 16 on the fly
        accsk.solve_points(_dev(torch, np.zeros((30, 17), np.float32), torch.float32),
                           _dev(torch, np.zeros((50, 17), np.float32), torch.float32), aa, bb, 1e-2, on_the_fly=True)
    assert e.value.status == accsk.SHAPE


@pytest.mark.parametrize("n,m", [(200, 300), (150, 2600)])
@pytest.mark.parametrize("method", [0, 1])
def test_on_the_fly_small_eps_fallback(torch_gpu, method, n, m):
    """eps = 1e-4 on unit-cube points: early steps have columns with almost no
    mass (exact column sweep), later steps the carried shifts; parity at tol.
    m = 2600 spreads the exact sweep's maximum and sum passes over two whole
    column chunks of the matrix-core sweeps and a ragged third."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _points(8, n, m, 3, 0)
    rng = np.random.default_rng(9)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    raw = O.cost_points(0, X, Y, 1.0)
    s = float(raw.max())
    eps = 1e-4
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps, cost_scale=s,
                                   on_the_fly=True, method=method, max_iter=400000)
    torch.cuda.synchronize()
    r = res[0]
    C = raw / s
    an, bn = a / a.sum(), b / b.sum()
    ev = O.evaluate(C, eps, an, bn, f.cpu().numpy(), g.cpu().numpy())
    print("eps 1e-4 method", method, n, m, "It", r["iters"], "fallback", r["fallback_steps"], "err", ev["err"], flush=True)
    assert r["converged"] == 1 and ev["err"] <= 1e-6 * 1.0001 and r["fallback_steps"] >= 1
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * eps + 1e-12 * abs(ev["dual"])


@pytest.mark.parametrize("d,split", [(2, 0), (33, 3)])
def test_blocks_without_rows_on_reused_workspace(torch_gpu, d, split):
    """40000 rows over 256 blocks of 160 rows leave the last six blocks without rows; their
    column partials must still be written (as zeros) every step.  The second of two identical
    solves runs on workspace the first one left dirty: it must converge and equal the first
    bit for bit (d = 2: FP64 matrix-core sweeps; d = 33: BF16 split-3 sweeps)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    n, m, eps = 40000, 40, 2e-2
    X, Y = _points(31 + d, n, m, d, 0)
    rng = np.random.default_rng(32)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d)
    args = [_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), _dev(torch, a, torch.float64),
            _dev(torch, b, torch.float64), eps]
    print("case blocks without rows, d", d, flush=True)
    outs = []
    for _ in range(2):
        f, g, res = accsk.solve_points(*args, cost_scale=s, split=split, on_the_fly=True)
        torch.cuda.synchronize()
        outs.append((f, g, res[0]))
        assert res[0]["converged"] == 1, res[0]
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2]["iters"] == outs[1][2]["iters"]
