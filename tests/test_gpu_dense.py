"""GPU parity of the dense explicit-cost solver against the FP64 oracle.

Tolerances (written here, derived from the arithmetic of the kernels):
* The kernel forms every exponent argument in FP64 and sums FP32 exp2 terms
  (pairwise per thread, FP64 across lanes and blocks), so each row/column
  log-sum-exp carries a relative error of a few FP32 ulps (~1e-7).  At the
  returned potentials the FP64 two-sided marginal error must therefore stay
  within tol (1e-6) plus that noise: we require err_fp64 <= tol.
* Stopping iteration: checked against the oracle's FP64 error trace of the
  same iteration (tests/_stopcheck.py): at the GPU's stop the oracle's error
  is below the threshold tol*(1 - 1/16) up to the GPU's 1.5e-7 error noise,
  and above it (same slack) at every earlier iterate.
* EOT value: both sides stop within tol of the optimum; the dual value is
  1-Lipschitz in the plan's L1 distance times max C, so they must agree to
  2*tol*max(C) + 1e-9 relative.
* Iterates at a fixed iteration count (tol = 0): the potentials in eps units
  (g/eps) agree to 1e-5 absolute after 30 steps.
"""
import numpy as np
import pytest

from oracle import oracle as O

from _stopcheck import check_stop
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu

from _stopcheck import STOP  # noqa: E402


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _solve_both(torch, C32, a, b, eps, tol, method, max_iter=20000, **kw):
    from paper_2605_30267_amd import accsk
    Cd = _dev(torch, C32, torch.float32)
    f, g, r = accsk.solve_dense(Cd, _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps,
                                tol=tol, method=method, max_iter=max_iter, **kw)
    torch.cuda.synchronize()
    o = O.solve(C32.astype(np.float64), a, b, eps, tol=tol * STOP, max_iter=max_iter,
                method=O.ACC if method == accsk.ACC else O.SINKHORN,
                mu0=kw.get("mu0") or accsk.default_params().mu0,
                m0=kw.get("m0") or accsk.default_params().m0,
                w_rule=kw.get("w_rule") if kw.get("w_rule") is not None else accsk.default_params().w_rule)
    o["method"] = O.ACC if method == accsk.ACC else O.SINKHORN
    return f.cpu().numpy(), g.cpu().numpy(), r, o


def _defaults():
    from paper_2605_30267_amd import accsk
    return accsk.default_params()


def _check(C32, a, b, eps, tol, fg, r, o, name):
    f, g = fg
    C = C32.astype(np.float64)
    an, bn = a / a.sum(), b / b.sum()
    ev = O.evaluate(C, eps, an, bn, f, g)
    print(name, "gpu It", r["iters"], "oracle It", o["iters"], "fp64 err", ev["err"], "gpu err",
          r["marginal_err"], "fallback", r["fallback_steps"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1
    assert ev["err"] <= tol, ev
    dp = _defaults()
    check_stop(C, an, bn, eps, tol, o["method"], r["iters"], dp.mu0, dp.m0, dp.w_rule)
    assert r["sinkhorn_steps"] == r["iters"] + 1
    # dual value at the returned potentials vs the oracle's at its own
    evo = O.evaluate(C, eps, an, bn, o["f"], o["g"])
    scale = 2 * tol * C.max() + 1e-9 * abs(evo["dual"])
    assert abs(r["eot_value"] - ev["dual"]) <= 1e-12 * abs(ev["dual"]) + 1e-15
    assert abs(ev["dual"] - evo["dual"]) <= scale
    assert abs(r["transport_cost"] - ev["cost"]) <= 1e-9 * abs(ev["cost"]) + 1e-13
    # gauge: g centred
    assert abs(g.mean()) <= 1e-12 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("method", [0, 1])
def test_small_uniform(torch_gpu, method):
    p = W.small_uniform()
    print("case small_uniform method", method, flush=True)
    f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], p["eps"], 1e-6, method)
    _check(p["C32"], p["a"], p["b"], p["eps"], 1e-6, (f, g), r, o, "small_uniform")


@pytest.mark.parametrize("n,m,eps,seed", [(37, 301, 1e-2, 11), (1000, 700, 3e-3, 12), (1, 1, 1e-2, 13),
                                          (5, 3000, 1e-2, 14), (200, 4097, 1e-2, 15), (3, 8192, 5e-2, 16),
                                          (513, 64, 1e-3, 17)])
@pytest.mark.parametrize("method", [0, 1])
def test_ragged_shapes(torch_gpu, n, m, eps, seed, method):
    p = W.random_dense(seed, n, m, eps=eps, a_kind="dirichlet")
    print("case ragged", n, m, eps, seed, method, flush=True)
    f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], eps, 1e-6, method)
    _check(p["C32"], p["a"], p["b"], eps, 1e-6, (f, g), r, o, "ragged %dx%d" % (n, m))


@pytest.mark.parametrize("method", [0, 1])
def test_fixed_iterates_match(torch_gpu, method):
    """tol = 0 forces max_iter steps: compare the iterates themselves."""
    p = W.random_dense(21, 300, 260, eps=1e-2)
    print("case fixed_iterates", method, flush=True)
    f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], 1e-2, 1e-300, method, max_iter=30)
    assert r["status"] == 4 and r["iters"] == 30 and o["iters"] == 30
    assert np.max(np.abs(g - o["g"])) / 1e-2 <= 1e-5
    assert np.max(np.abs(f - o["f"])) / 1e-2 <= 1e-5


def test_w_rules_and_homotopy(torch_gpu):
    # above 256 x 256 entries: the cooperative solver (smaller problems run on one workgroup)
    p = W.random_dense(22, 320, 300, eps=3e-3)
    for rule in (0, 1):
        for mu0, m0 in ((0.5, 1), (0.1, 10), (0.9, 2)):
            print("case homotopy", rule, mu0, m0, flush=True)
            f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], 3e-3, 1e-300, 1, max_iter=40,
                                     mu0=mu0, m0=m0, w_rule=rule)
            assert np.max(np.abs(g - o["g"])) / 3e-3 <= 1e-5, (rule, mu0, m0)


def test_small_eps_fallback(torch_gpu):
    """eps = 1e-4: early columns receive almost no mass, exercising the exact column pass
    of the cooperative solver (the one-workgroup solver's is covered by the batch tests)."""
    p = W.random_dense(23, 300, 300, eps=1e-4)
    print("case small eps", flush=True)
    f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], 1e-4, 1e-6, 1)
    _check(p["C32"], p["a"], p["b"], 1e-4, 1e-6, (f, g), r, o, "eps1e-4")
    assert r["fallback_steps"] >= 1


def test_deterministic(torch_gpu):
    from paper_2605_30267_amd import accsk
    torch = torch_gpu
    p = W.random_dense(24, 640, 900, eps=1e-2)
    Cd = _dev(torch, p["C32"], torch.float32)
    a, b = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    f1, g1, r1 = accsk.solve_dense(Cd, a, b, 1e-2)
    f2, g2, r2 = accsk.solve_dense(Cd, a, b, 1e-2)
    torch.cuda.synchronize()
    r1.pop("kernel_ms")
    r2.pop("kernel_ms")
    assert torch.equal(f1, f2) and torch.equal(g1, g2) and r1 == r2


def test_errors(torch_gpu):
    from paper_2605_30267_amd import accsk
    torch = torch_gpu
    p = W.random_dense(25, 64, 64)
    Cd = _dev(torch, p["C32"], torch.float32)
    a, b = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    bad = a.clone()
    bad[3] = 0.0
    _, _, r = accsk.solve_dense(Cd, bad, b, 1e-2, raise_on_error=False)
    assert r["status"] == accsk.INVALID_ARG
    bad[3] = float("nan")
    _, _, r = accsk.solve_dense(Cd, bad, b, 1e-2, raise_on_error=False)
    assert r["status"] == accsk.NONFINITE
    Cn = Cd.clone()
    Cn[5, 7] = float("nan")
    _, _, r = accsk.solve_dense(Cn, a, b, 1e-2, raise_on_error=False)
    assert r["status"] == accsk.NONFINITE
    _, _, r = accsk.solve_dense(Cd, a, b, 1e-2, tol=1e-300, max_iter=3, raise_on_error=False)
    assert r["status"] == accsk.NOT_CONVERGED and r["iters"] == 3
    _, _, r = accsk.solve_dense(Cd, a, b, -1.0, raise_on_error=False)
    assert r["status"] == accsk.INVALID_ARG


def test_plan_and_eval(torch_gpu):
    from paper_2605_30267_amd import accsk
    torch = torch_gpu
    p = W.small_uniform(seed=31, n=200, m=150)
    Cd = _dev(torch, p["C32"], torch.float32)
    a, b = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    f, g, r = accsk.solve_dense(Cd, a, b, p["eps"])
    P = accsk.plan_dense(Cd, f, g, p["eps"], row0=17, rows=50).cpu().numpy()
    ev = accsk.eval_dense(Cd, a, b, f, g, p["eps"])
    fh, gh = f.cpu().numpy(), g.cpu().numpy()
    Po = O.plan(p["C32"].astype(np.float64), p["eps"], fh, gh, row0=17, rows=50)
    big = Po > 1e-30  # FP32 output: below this the value may be denormal or zero
    assert np.max(np.abs(P[big] - Po[big]) / Po[big]) <= 2e-6
    assert np.all(P[~big] <= 2e-30)
    evo = O.evaluate(p["C32"].astype(np.float64), p["eps"], p["a"], p["b"], fh, gh)
    for k in ("row_err", "col_err"):
        assert abs(ev[k] - evo[k]) <= 1e-12 + 1e-9 * evo[k]
    for k in ("dual", "cost", "mass"):
        assert abs(ev[k] - evo[k]) <= 1e-12 * max(1.0, abs(evo[k]))


@pytest.mark.parametrize("m", [2048, 3000, 4097, 8192])
def test_exact_column_pass_wide(torch_gpu, m):
    """eps = 1e-4 with 2 % of the columns out of every row's reach at the start
    (column sums near 2^-7000): the exact column pass runs in each workgroup-rows
    instantiation of the cooperative solver (m = 2048: 512 threads, four rows per
    batch; 3000: 1024 threads, two rows; 4097 and 8192: 1024 threads, two column
    groups per thread, with and without 16-byte loads).  FP64 two-sided error of
    the result <= tol, dual value, stopping iterate against the oracle."""
    p = W.outlier_columns(51, 600, m, eps=1e-4)
    print("case outlier columns 600 x", m, flush=True)
    f, g, r, o = _solve_both(torch_gpu, p["C32"], p["a"], p["b"], 1e-4, 1e-6, 1)
    print("  It", r["iters"], "fallback", r["fallback_steps"], "oracle It", o["iters"], flush=True)
    _check(p["C32"], p["a"], p["b"], 1e-4, 1e-6, (f, g), r, o, "outlier%d" % m)
    assert r["fallback_steps"] >= 1


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4])
def test_gmm_full_size(torch_gpu, eps):
    """n = m = 8192: KKT in FP64, sampled exact row solves, dual value, both methods."""
    from paper_2605_30267_amd import accsk
    torch = torch_gpu
    p = W.gmm_dense(eps=eps)
    Cd = _dev(torch, p["C32"], torch.float32)
    a, b = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    C = p["C32"].astype(np.float64)
    for method in (1, 0):
        print("case gmm 8192 eps", eps, "method", method, flush=True)
        f, g, r = accsk.solve_dense(Cd, a, b, eps, method=method, max_iter=200000)
        torch.cuda.synchronize()
        fh, gh = f.cpu().numpy(), g.cpu().numpy()
        ev = O.evaluate(C, eps, p["a"], p["b"], fh, gh)
        print("  It", r["iters"], "fp64 err", ev["err"], "gpu err", r["marginal_err"], "fallback",
              r["fallback_steps"], flush=True)
        assert r["converged"] == 1 and ev["err"] <= 1e-6
        assert abs(r["eot_value"] - ev["dual"]) <= 1e-12 * abs(ev["dual"])
        rng = np.random.default_rng(7)
        rows = np.sort(rng.choice(C.shape[0], 64, replace=False))
        # exact row solve of the oracle on the sampled rows at the GPU's g (eq:u-update)
        st = O.sstep(C[rows], eps, p["a"][rows], p["b"], gh / eps)
        assert np.max(np.abs(st["u"] * eps - fh[rows])) / eps <= 1e-6
