"""Point-cloud solves with the cost formed on the fly on the matrix cores
(16 < d <= 128, split 2 or 3): the tiled solver's row and column sweeps compute
x_i . y_j from v_mfma_f32_16x16x32_bf16 on BF16 pieces of X and Y and never
store C (Sec. 5 costs, eq:P-from-dual).

Tolerance (derived from the arithmetic, written here): the solve converges on
the cost C~ = C + dC its tiles produce, to the library's stop rule.  On the
exact FP64 cost its plan changes entry by entry by the factor exp(dC/eps), so
the exact-cost L1 marginal error is at most tol + 2 max|dC| / eps (rows and
columns).  dC = c_s e / s with c_s = 2 (squared Euclidean: |x|^2 + |y|^2 - 2 x.y,
norms in FP64) or 1 (cosine), and the cross-term error
  e <= beta * sum_k |x_k| |y_k|,
  beta = 2^-24 (pieces dropped and residual of the 3-piece split)
       + (6 K/32 + 1) 2^-24 (FP32 accumulation: one rounding per product
         instruction into a sum bounded by sum_k |x_k||y_k|, K the padded depth),
with 2^-16 for the residual of a 2-piece split.  A wrong operand or result
layout gives errors of the order of C itself.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _clouds(seed, n, m, d, kind):
    rng = np.random.default_rng(seed)
    if kind == 1:
        return W.unit_rows(rng, n, d).astype(np.float32), W.unit_rows(rng, m, d).astype(np.float32)
    X = rng.standard_normal(size=(n, d)).astype(np.float32)
    Y = (rng.standard_normal(size=(m, d)) + 0.25).astype(np.float32)
    return X, Y


def _beta(d, split):
    K = 32 * math.ceil(d / 32)
    K = 32 if K <= 32 else (64 if K <= 64 else 128)
    products = 6 if split == 3 else 3
    rep = 2.0 ** -24 if split == 3 else 2.0 ** -16
    return rep + (products * K // 32 + 1) * 2.0 ** -24


def _cost_err_bound(X, Y, kind, s, split):
    cross = np.abs(X.astype(np.float64)) @ np.abs(Y.astype(np.float64)).T
    return (2.0 if kind == 0 else 1.0) * _beta(X.shape[1], split) * float(cross.max()) / s


@pytest.mark.parametrize("kind,n,m,d,eps,split", [
    (0, 300, 500, 64, 1e-2, 3),     # one round, ragged rows and columns
    (1, 700, 257, 100, 3e-3, 3),    # cosine, K padded to 128
    (0, 2000, 1000, 17, 1e-2, 3),   # K = 32
    (0, 257, 130, 128, 5e-3, 2),    # 2-piece split
    (0, 40000, 50, 33, 2e-2, 3),    # 157 rows per block: two rounds per wave
    (1, 1, 1, 20, 1e-1, 3),         # one entry
])
def test_on_the_fly_mfma(torch_gpu, kind, n, m, d, eps, split):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(100 + n + d, n, m, d, kind)
    rng = np.random.default_rng(n * 7 + m)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = 2.0 * d if kind == 0 else 1.0
    print("case mfma on the fly", kind, n, m, d, eps, split, flush=True)
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps, kind=kind,
                                   cost_scale=s, split=split, on_the_fly=True, max_iter=200000)
    torch.cuda.synchronize()
    r = res[0]
    an, bn = a / a.sum(), b / b.sum()
    ev = O.evaluate_points(kind, X, Y, s, eps, an, bn, f.cpu().numpy(), g.cpu().numpy())
    dC = _cost_err_bound(X, Y, kind, s, split)
    bound = 1e-6 + 2.0 * dC / eps
    print("  It", r["iters"], "fallback", r["fallback_steps"], "exact-cost err", ev["err"], "bound", bound,
          "max|dC|", dC, flush=True)
    assert r["status"] == 0 and r["converged"] == 1, r
    assert ev["err"] <= bound
    # <C,P> at the returned potentials: FP64 cost, FP32 exponentials of FP64 arguments, FP64 sums
    assert abs(r["transport_cost"] - ev["cost"]) <= 1e-6 * abs(ev["cost"]) + 1e-13
    assert abs(float(g.mean())) <= 1e-9 * max(1.0, float(g.abs().max()))


def test_on_the_fly_mfma_exact_column_sweep(torch_gpu):
    """2% of the Y points moved far from every X point: at eps = 1e-3 their columns receive
    almost no mass in the first steps (column sums below 2^-64), which the exact column
    sweep (per-block column maximum, then the sums) redoes; parity as above."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    n, m, d, eps = 500, 400, 48, 1e-3
    X, Y = _clouds(77, n, m, d, 0)
    Y[: m // 50] += 3.0
    rng = np.random.default_rng(78)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = 2.0 * d
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps, cost_scale=s,
                                   split=3, on_the_fly=True, max_iter=200000)
    torch.cuda.synchronize()
    r = res[0]
    ev = O.evaluate_points(0, X, Y, s, eps, a / a.sum(), b / b.sum(), f.cpu().numpy(), g.cpu().numpy())
    bound = 1e-6 + 2.0 * _cost_err_bound(X, Y, 0, s, 3) / eps
    print("exact column sweep: It", r["iters"], "fallback", r["fallback_steps"], "err", ev["err"], "bound", bound,
          flush=True)
    assert r["converged"] == 1 and r["fallback_steps"] >= 1
    assert ev["err"] <= bound


def test_on_the_fly_mfma_against_materialized(torch_gpu):
    """The same split-3 solve with C built by the matrix cores and stored: both solve
    perturbations of one cost, so their dual values at the returned potentials agree to
    the sum of the two cost errors (and the stored path's own 2^-20 B bound)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    n, m, d, eps = 1024, 1536, 64, 5e-3
    p = W.gaussian_batch(seed=17, batch=1, n=n, m=m, d=d, eps=eps)
    X, Y = p["X"][0], p["Y"][0]
    args = [_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), _dev(torch, p["a"][0], torch.float64),
            _dev(torch, p["b"][0], torch.float64), eps]
    f1, g1, r1 = accsk.solve_points(*args, cost_scale=p["scale"], split=3, on_the_fly=True)
    f2, g2, r2 = accsk.solve_points(*args, cost_scale=p["scale"], split=3)
    torch.cuda.synchronize()
    an, bn = p["a"][0] / p["a"][0].sum(), p["b"][0] / p["b"][0].sum()
    e1 = O.evaluate_points(0, X, Y, p["scale"], eps, an, bn, f1.cpu().numpy(), g1.cpu().numpy())
    e2 = O.evaluate_points(0, X, Y, p["scale"], eps, an, bn, f2.cpu().numpy(), g2.cpu().numpy())
    B = (np.linalg.norm(X.astype(np.float64), axis=1).max() ** 2 +
         np.linalg.norm(Y.astype(np.float64), axis=1).max() ** 2) / p["scale"]
    dC = _cost_err_bound(X, Y, 0, p["scale"], 3) + 2.0 ** -20 * B
    print("on the fly It", r1[0]["iters"], "err", e1["err"], "dual", e1["dual"], "| stored It", r2[0]["iters"],
          "err", e2["err"], "dual", e2["dual"], flush=True)
    assert r1[0]["converged"] == 1 and r2[0]["converged"] == 1
    # each dual value is within (tol + 2 max|dC|/eps) * max C of the exact optimum
    cmax = float(O.cost_points(0, X, Y, p["scale"]).max())
    assert abs(e1["dual"] - e2["dual"]) <= 2 * (1e-6 + 2 * dC / eps) * cmax + 1e-9 * abs(e2["dual"])
