"""Pins of the oracle's boundedness monitor (App. B, Theorem thm:condition-boundedness,
eq:D, and the shifted Lyapunov function of the theorem's proof).

* The metric D_jj = b_j (e^p - 1)/p (p = log(c_j/b_j)) and D_phi*(0, c - b) =
  sum_j (c_j - b_j - b_j p_j) against 50-digit decimal arithmetic on the same
  binary inputs, across the series switch at |p| = 1e-2, at c = b and far from it.
* On a separable cost C_ij = alpha_i + beta_j everything has a closed form: the
  column sums at the exact row solve are c = softmax(x - beta), Sinkhorn(x) is
  the constant x* = centre(log b + beta), and w is recovered from consecutive
  iterates (x_{k+1} = (w_k + x*)/(1 + alpha)).  The oracle's per-iterate
  monitor rows (lhs1, rhs1, lhs2, rhs2, E) are recomputed from its x trace
  through those closed forms and the decimal metric, for both hand-off rules,
  and so are its violation counts.  A wrong pairing of iterates, a wrong v
  (w/alpha - x), a missed stage rebase or a wrong constant fails here.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import oracle as O

getcontext().prec = 50


def _dec_metric(c, b):
    """D and the D_phi*(0, c - b) term of one column in 50-digit arithmetic."""
    C, B = Decimal(float(c)), Decimal(float(b))
    if C == B:
        return float(B), 0.0
    lp = (C / B).ln()
    return float((C - B) / lp), float(C - B - B * lp)


@pytest.mark.parametrize("rel", [0.0, 1e-12, -3e-9, 2e-6, -5e-4, 9e-4, -1.1e-3, 2e-3, -9e-3, 1.3e-2, 0.05, -0.3, 3.0, 99.0])
def test_metric_against_decimal(rel):
    rng = np.random.default_rng(7)
    b = rng.uniform(1e-4, 1e-1, size=16)
    c = b * (1.0 + rel * rng.uniform(0.5, 1.0, size=16))
    D, K = O.cond_metric(c, b)
    for j in range(16):
        d_ref, k_ref = _dec_metric(c[j], b[j])
        assert abs(D[j] - d_ref) <= 1e-14 * abs(d_ref), (rel, j, D[j], d_ref)
        # K ~ b p^2 / 2: its FP64 value carries the rounding of c - b relative to b
        assert abs(K[j] - k_ref) <= 1e-13 * abs(k_ref) + 1e-17 * b[j], (rel, j, K[j], k_ref)


def _separable(seed, n, m):
    rng = np.random.default_rng(seed)
    al = rng.uniform(0, 1, n)
    be = rng.uniform(0, 1, m)
    a = rng.uniform(0.5, 1.5, n)
    b = rng.uniform(0.5, 1.5, m)
    return al, be, a / a.sum(), b / b.sum()


def _stages(mu0, m0, iters):
    """(alpha, mu) of the stage of every iterate 0..iters, and the iterates that end a stage."""
    ab, ends = [], set()
    mu, ms, k = mu0, m0, 0
    ab.append((math.sqrt(2 * mu), mu))  # iterate 0 belongs to the first stage
    while k < iters:
        for _ in range(ms):
            if k >= iters:
                break
            k += 1
            ab.append((math.sqrt(2 * mu), mu))
        if k < iters or len(ab) == iters + 1:
            ends.add(k)
        mu /= 2.0
        ms = int(math.floor(math.sqrt(2.0) * ms)) + 1
    return ab, ends


@pytest.mark.parametrize("w_rule", [O.W_LITERAL, O.W_Y_CONTINUOUS])
def test_monitor_trace_on_separable_cost(w_rule):
    n, m, eps = 7, 9, 1.0
    al, be, a, b = _separable(11, n, m)
    C = al[:, None] + be[None, :]
    mu0, m0 = 0.25, 3
    o = O.solve(C, a, b, eps, tol=1e-13, max_iter=60, mu0=mu0, m0=m0, w_rule=w_rule, trace=True, trace_x=True,
                conditions=True)
    It = o["iters"]
    assert It >= 12
    X = o["trace_x"]
    xstar = np.log(b) + be
    xstar -= xstar.mean()
    ab, ends = _stages(mu0, m0, It)

    def csum(x):
        z = x - be
        e = np.exp(z - z.max())
        return e / e.sum()

    def fval(x):
        z = x - be
        lse = z.max() + np.log(np.exp(z - z.max()).sum())
        return 1.0 - float(np.dot(a, np.log(a) + al)) + lse - float(np.dot(x, b))

    def metric(x):
        c = csum(x)
        out = [_dec_metric(c[j], b[j]) for j in range(m)]
        return c - b, np.array([t[0] for t in out]), np.array([t[1] for t in out]).sum()

    # w handed to the x update that made iterate k+1, and w_k before any stage rescale
    w_hand = [(1.0 + ab[k + 1][0]) * X[k + 1] - xstar for k in range(It)]
    w_pre = []
    for k in range(It):
        if k in ends and w_rule == O.W_Y_CONTINUOUS:
            w_pre.append(w_hand[k] * ab[k][0] / ab[k + 1][0])
        else:
            w_pre.append(w_hand[k])
    tc = o["trace_cond"]
    n1 = n2 = nl = 0
    E_base = None
    for k in range(It - 1):  # pairs (k, k+1); the last iterate's w is not in the trace
        alpha, mu = ab[k + 1]
        xi0, D0, K0 = metric(X[k])
        xi1, D1, K1 = metric(X[k + 1])
        vb = w_hand[k] / alpha - X[k]
        vn = w_pre[k + 1] / alpha - X[k + 1]
        lhs1 = float(np.sum(xi0 ** 2 * D1 / D0 ** 2))
        rhs1 = (4 - alpha ** 2 - 2 * math.sqrt(alpha)) / (2 * alpha * (1 + alpha) ** 2) * K0
        lhs2 = float(np.sum(vb ** 2 * (D1 - D0)))
        vd = float(np.sum(vn ** 2 * D1))
        rhs2 = alpha ** 1.5 * vd
        theta = (0.5 + alpha) / (1 + alpha)
        E1 = fval(X[k + 1]) + 0.5 * mu * vd - theta / (1 + alpha) * K1
        row = tc[k + 1]
        for got, ref in zip(row, (lhs1, rhs1, lhs2, rhs2, E1)):
            assert abs(got - ref) <= 1e-9 * abs(ref) + 1e-13, (k, row, (lhs1, rhs1, lhs2, rhs2, E1))
        E0 = fval(X[k]) + 0.5 * mu * float(np.sum(vb ** 2 * D0)) - theta / (1 + alpha) * K0
        n1 += not lhs1 < rhs1
        n2 += not lhs2 < rhs2
        nl += E1 > E0 + 1e-8 + 1e-12 * abs(fval(X[k + 1])) + 1e-6 * (0.5 * mu * vd + float(np.abs(xi1).sum()))
        E_base = E1
    assert E_base is not None
    # counts over the pairs recomputed above (the oracle also counts the last pair)
    c1, c2, cl = o["cond_counts"]
    assert n1 <= c1 <= n1 + 1 and n2 <= c2 <= n2 + 1 and nl <= cl <= nl + 1, (o["cond_counts"], n1, n2, nl)


def test_monitor_counts_shape_of_theory():
    """Condition 1 needs (4 - alpha^2 - 2 sqrt(alpha)) / (2 alpha (1+alpha)^2) above about 2 (its left
    side is about ||xi||^2_{D^-1} ~ 2 K): it fails in the first homotopy stages (alpha = 0.71, 0.5)
    and holds once alpha is small; Sinkhorn is not monitored."""
    rng = np.random.default_rng(3)
    C = rng.uniform(0, 1, (40, 30))
    a = rng.uniform(0.5, 1.5, 40)
    b = rng.uniform(0.5, 1.5, 30)
    o = O.solve(C, a, b, 1e-2, tol=1e-10, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS, conditions=True, trace=True)
    t = o["trace_cond"]
    ab, _ = _stages(0.25, 5, o["iters"])
    late = [k for k in range(1, o["iters"] + 1) if ab[k][0] < 0.2]
    early = [k for k in range(1, o["iters"] + 1) if ab[k][0] > 0.6]
    assert late and early
    assert all(t[k, 0] < t[k, 1] for k in late)
    assert all(not t[k, 0] < t[k, 1] for k in early)
    s = O.solve(C, a, b, 1e-2, tol=1e-10, method=O.SINKHORN, conditions=True)
    assert s["cond_counts"] == [-1, -1, -1]
