"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it follows.  None of them re-types the oracle's
own formulas: they use closed forms, an exact LP, brute-force minimization,
invariances, the inequalities of App. A, and finite differences, chosen so that
a dropped term, a wrong sign or index, or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.optimize import linprog, minimize

from oracle import oracle as O


def _rng(seed):
    return np.random.default_rng(seed)


def _problem(seed, n, m, kind="uniform"):
    r = _rng(seed)
    C = r.uniform(0.0, 1.0, size=(n, m))
    a = r.uniform(0.5, 1.5, size=n)
    b = r.uniform(0.5, 1.5, size=m)
    return C, a / a.sum(), b / b.sum()


def _plan(C, eps, f, g):
    return np.exp((f[:, None] + g[None, :] - C) / eps)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("method", [O.SINKHORN, O.ACC])
def test_separable_cost_closed_form(method):
    """C_ij = alpha_i + beta_j: the plan is a b^T and the EOT value is known.

    With a separable cost the entropic problem decouples (eq:EOT): P* = a b^T,
    value = <alpha,a> + <beta,b> + eps * sum_ij a_i b_j (log(a_i b_j) - 1).
    Plain Sinkhorn reaches it after one column update (eq:v-update).
    """
    r = _rng(1)
    n, m, eps = 7, 5, 0.05
    al, be = r.uniform(0, 1, n), r.uniform(0, 1, m)
    C = al[:, None] + be[None, :]
    a, b = r.dirichlet(np.ones(n)), r.dirichlet(np.ones(m))
    out = O.solve(C, a, b, eps, tol=1e-13, method=method, mu0=0.5, m0=1, w_rule=O.W_Y_CONTINUOUS)
    assert out["converged"]
    P = _plan(C, eps, out["f"], out["g"])
    np.testing.assert_allclose(P, np.outer(a, b), rtol=1e-10, atol=1e-15)
    ab = np.outer(a, b)
    val = al @ a + be @ b + eps * np.sum(ab * (np.log(ab) - 1.0))
    ev = O.evaluate(C, eps, a, b, out["f"], out["g"])
    assert abs(ev["dual"] - val) <= 1e-12
    assert abs(ev["cost"] - (al @ a + be @ b)) <= 1e-12
    if method == O.SINKHORN:
        assert out["iters"] == 1


@pytest.mark.parametrize("seed", range(5))
def test_two_by_two_closed_form(seed):
    """2x2: P11 = p solves (1-q)p^2 + (a2 - b1 + q(a1+b1))p - q a1 b1 = 0.

    From eq:P-from-dual, P11 P22 / (P12 P21) = exp(-(C11+C22-C12-C21)/eps) = q,
    and the marginals fix P in terms of p.
    """
    r = _rng(100 + seed)
    C = r.uniform(0, 1, size=(2, 2))
    a = r.dirichlet([1, 1])
    b = r.dirichlet([1, 1])
    eps = [1.0, 0.3, 0.1, 0.05, 0.02][seed]
    q = math.exp(-(C[0, 0] + C[1, 1] - C[0, 1] - C[1, 0]) / eps)
    A2, B2, C2 = 1 - q, a[1] - b[0] + q * (a[0] + b[0]), -q * a[0] * b[0]
    lo, hi = max(0.0, b[0] - a[1]), min(a[0], b[0])
    if abs(A2) < 1e-14:
        p = -C2 / B2
    else:
        roots = np.roots([A2, B2, C2]).real
        p = [x for x in roots if lo - 1e-14 <= x <= hi + 1e-14][0]
    out = O.solve(C, a, b, eps, tol=1e-14, method=O.ACC, mu0=0.5, m0=2, max_iter=100000,
                  w_rule=O.W_Y_CONTINUOUS)
    assert out["converged"]
    P = _plan(C, eps, out["f"], out["g"])
    expect = np.array([[p, a[0] - p], [b[0] - p, a[1] - b[0] + p]])
    np.testing.assert_allclose(P, expect, rtol=1e-9, atol=1e-14)


def _acc_closed_form_iterates(xstar, mu0, m0, w_rule, K):
    """Acc iterates when Sinkhorn(x) == x* for every x (separable cost).

    Within a stage with step alpha, the errors e_x = x - x*, e_w = w - alpha x*
    obey e_x,k+1 = e_w,k/(1+alpha), e_w,k+1 = rho e_w,k,
    rho = (alpha^2 + alpha - 1)/(1 + alpha)^2 (solved recurrence of Algorithm A2MD).
    Across stages (Algorithm A2MD-homotopy) w is carried (LITERAL) or rescaled
    by alpha_new/alpha_old (Y_CONTINUOUS).
    """
    xs = [np.zeros_like(xstar)]
    w = np.zeros_like(xstar)
    mu, mst, k = mu0, m0, 0
    while k < K:
        al = math.sqrt(2 * mu)
        rho = (al * al + al - 1) / (1 + al) ** 2
        ew0 = w - al * xstar
        for j in range(mst):
            if k >= K:
                break
            xs.append(xstar + (rho ** j) * ew0 / (1 + al))
            k += 1
        w = al * xstar + (rho ** min(mst, j + 1)) * ew0
        mu_new = mu / 2
        if w_rule == O.W_Y_CONTINUOUS:
            w = w * math.sqrt(2 * mu_new) / al
        mu = mu_new
        mst = int(math.floor(math.sqrt(2) * mst)) + 1
    return np.array(xs)


@pytest.mark.parametrize("w_rule", [O.W_LITERAL, O.W_Y_CONTINUOUS])
@pytest.mark.parametrize("mu0,m0", [(0.5, 1), (0.3, 3), (0.9, 2)])
def test_acc_recurrence_closed_form(w_rule, mu0, m0):
    """Separable cost: Sinkhorn(x) = center(log b + beta/eps) for all x, so the
    accelerated recurrence has the closed form above; the oracle must follow it."""
    r = _rng(7)
    n, m, eps = 6, 9, 0.2
    al, be = r.uniform(0, 1, n), r.uniform(0, 1, m)
    C = al[:, None] + be[None, :]
    a, b = r.dirichlet(np.ones(n)), r.dirichlet(np.ones(m))
    K = 40
    out = O.solve(C, a, b, eps, tol=1e-300, max_iter=K, method=O.ACC, mu0=mu0, m0=m0, w_rule=w_rule,
                  trace_x=True)
    xstar = np.log(b) + be / eps
    xstar -= xstar.mean()
    ref = _acc_closed_form_iterates(xstar, mu0, m0, w_rule, K)
    np.testing.assert_allclose(out["trace_x"], ref, rtol=1e-12, atol=1e-12 * np.abs(xstar).max())


# ---------------------------------------------------------------------------
# The second form of the accelerated scheme
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [0.5, 0.2, 0.05])
def test_algorithm_equals_xy_scheme(mu):
    """Algorithm A2MD (w = alpha y) and eq:scheme with explicit y, written with
    the mirror map log(1 + xi./b) of Sec. 3, give the same x iterates."""
    C, a, b = _problem(3, 12, 9)
    eps, K = 0.05, 25
    out = O.solve(C, a, b, eps, tol=1e-300, max_iter=K, method=O.ACC, mu0=mu, m0=10 ** 6, trace_x=True)
    xs = O.scheme_xy(C, eps, a, b, mu, K)
    np.testing.assert_allclose(out["trace_x"], xs, rtol=1e-10, atol=1e-10)


def test_sinkhorn_equals_mirror_step():
    """Sec. 3 eq:md-general: v - grad phi*(grad f(v)) = v + log(b ./ c_P) is the
    Sinkhorn v-update; after centring it equals the oracle's Sinkhorn(v)."""
    C, a, b = _problem(4, 10, 8)
    eps = 0.1
    x = _rng(5).normal(size=8)
    x -= x.mean()
    st = O.sstep(C, eps, a, b, x)
    p = O.mirror_step_p(C, eps, a, b, x)
    np.testing.assert_allclose(st["S"], x - p, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# LP, KKT, brute force
# ---------------------------------------------------------------------------

def _ot_lp(C, a, b):
    n, m = C.shape
    Aeq = np.zeros((n + m, n * m))
    for i in range(n):
        Aeq[i, i * m:(i + 1) * m] = 1
    for j in range(m):
        Aeq[n + j, j::m] = 1
    res = linprog(C.ravel(), A_eq=Aeq, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed,n,m", [(11, 6, 6), (12, 8, 5), (13, 10, 10)])
def test_lp_gap_bound(seed, n, m):
    """0 <= <C,P^eps> - OT <= eps log(nm) (Sec. 4, discussion on complexity),
    and the gap shrinks as eps decreases."""
    C, a, b = _problem(seed, n, m)
    ot = _ot_lp(C, a, b)
    gaps = []
    for eps in (0.1, 0.03, 0.01, 0.003):
        out = O.solve(C, a, b, eps, tol=1e-11, method=O.ACC, mu0=0.1, m0=10, w_rule=O.W_Y_CONTINUOUS,
                      max_iter=200000)
        ev = O.evaluate(C, eps, a, b, out["f"], out["g"])
        gap = ev["cost"] - ot
        assert -1e-9 <= gap <= eps * math.log(n * m) + 1e-9
        gaps.append(gap)
    assert gaps[-1] < gaps[0]


def test_kkt_independent_marginals():
    """Any (f, g) whose plan has the marginals a, b is the EOT optimum (eq:grad-F);
    marginals are recomputed here with numpy, independently of the oracle."""
    C, a, b = _problem(21, 30, 25)
    for eps in (0.5, 0.05, 0.01):
        for method in (O.SINKHORN, O.ACC):
            out = O.solve(C, a, b, eps, tol=1e-10, method=method, mu0=0.1, m0=10, w_rule=O.W_Y_CONTINUOUS)
            P = _plan(C, eps, out["f"], out["g"])
            assert np.abs(P.sum(1) - a).sum() + np.abs(P.sum(0) - b).sum() < 1e-10


def test_brute_force_dual():
    """Maximize the EOT dual <f,a> + <g,b> - eps sum exp((f_i+g_j-C_ij)/eps)
    (eq:dual-obj) with a generic quasi-Newton method; same optimum."""
    C, a, b = _problem(22, 4, 3)
    eps = 0.2

    def negdual(z):
        f, g = z[:4], z[4:]
        P = np.exp((f[:, None] + g[None, :] - C) / eps)
        val = f @ a + g @ b - eps * P.sum()
        grad = np.concatenate([a - P.sum(1), b - P.sum(0)])
        return -val, -grad

    res = minimize(negdual, np.zeros(7), jac=True, method="BFGS", options=dict(gtol=1e-13, maxiter=10000))
    out = O.solve(C, a, b, eps, tol=1e-13, method=O.SINKHORN)
    ev = O.evaluate(C, eps, a, b, out["f"], out["g"])
    assert abs(ev["dual"] - (-res.fun)) <= 1e-10
    Pb = np.exp((res.x[:4, None] + res.x[None, 4:] - C) / eps)
    np.testing.assert_allclose(_plan(C, eps, out["f"], out["g"]), Pb, atol=1e-7)


# ---------------------------------------------------------------------------
# Invariances
# ---------------------------------------------------------------------------

def test_invariances():
    """C + c leaves P unchanged and shifts the value by c; (C, eps) -> (sC, s eps)
    leaves P unchanged and scales the value by s; permuting rows permutes f."""
    C, a, b = _problem(31, 9, 7)
    eps = 0.05
    base = O.solve(C, a, b, eps, tol=1e-12, method=O.SINKHORN)
    Pb = _plan(C, eps, base["f"], base["g"])
    vb = O.evaluate(C, eps, a, b, base["f"], base["g"])["dual"]
    sh = O.solve(C + 0.7, a, b, eps, tol=1e-12, method=O.SINKHORN)
    np.testing.assert_allclose(_plan(C + 0.7, eps, sh["f"], sh["g"]), Pb, rtol=1e-9, atol=1e-14)
    assert abs(O.evaluate(C + 0.7, eps, a, b, sh["f"], sh["g"])["dual"] - (vb + 0.7)) <= 1e-11
    sc = O.solve(3.0 * C, a, b, 3.0 * eps, tol=1e-12, method=O.SINKHORN)
    np.testing.assert_allclose(_plan(3 * C, 3 * eps, sc["f"], sc["g"]), Pb, rtol=1e-9, atol=1e-14)
    assert abs(O.evaluate(3 * C, 3 * eps, a, b, sc["f"], sc["g"])["dual"] - 3 * vb) <= 1e-11
    perm = _rng(3).permutation(9)
    pr = O.solve(C[perm], a[perm], b, eps, tol=1e-12, method=O.SINKHORN)
    np.testing.assert_allclose(pr["f"], base["f"][perm], atol=1e-9)


def test_sinkhorn_and_acc_same_optimum():
    """Uniqueness of the optimum modulo the gauge (eq:Fc)."""
    C, a, b = _problem(41, 40, 30)
    eps = 0.02
    s = O.solve(C, a, b, eps, tol=1e-12, method=O.SINKHORN, max_iter=200000)
    acc = O.solve(C, a, b, eps, tol=1e-12, method=O.ACC, mu0=0.1, m0=10, w_rule=O.W_Y_CONTINUOUS)
    np.testing.assert_allclose(acc["g"], s["g"], atol=1e-9)
    np.testing.assert_allclose(acc["f"], s["f"], atol=1e-9)
    d1 = O.evaluate(C, eps, a, b, s["f"], s["g"])["dual"]
    d2 = O.evaluate(C, eps, a, b, acc["f"], acc["g"])["dual"]
    assert abs(d1 - d2) <= 1e-10 * abs(d1)


# ---------------------------------------------------------------------------
# Derivatives of the reduced objective
# ---------------------------------------------------------------------------

def test_grad_f_finite_differences():
    """grad f(v) = c_P(u(v), v) - b (eq:grad-f), checked by central differences
    of f(v) = 1 - <u(v),a> - <v,b> (Lemma coercivity)."""
    C, a, b = _problem(51, 8, 6)
    eps = 0.3
    v = _rng(2).normal(size=6) * 0.3
    st = O.sstep(C, eps, a, b, v)
    c = np.exp(v + st["ell"])
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (O.sstep(C, eps, a, b, v + e)["fval"] - O.sstep(C, eps, a, b, v - e)["fval"]) / (2 * h)
        assert abs(fd - (c[j] - b[j])) <= 1e-8


def test_hessian_finite_differences():
    """Hess f = diag(c_P) - P' diag(r_P)^{-1} P (eq:HessianL); its kernel is span{1}."""
    C, a, b = _problem(52, 7, 5)
    eps = 0.4
    v = _rng(3).normal(size=5) * 0.2
    st = O.sstep(C, eps, a, b, v)
    P = np.exp(st["u"][:, None] + v[None, :] - C / eps)
    H = np.diag(P.sum(0)) - P.T @ np.diag(1.0 / P.sum(1)) @ P
    h = 1e-5
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        cp = np.exp(v + e + O.sstep(C, eps, a, b, v + e)["ell"])
        cm = np.exp(v - e + O.sstep(C, eps, a, b, v - e)["ell"])
        np.testing.assert_allclose((cp - cm) / (2 * h), H[:, j], atol=1e-8)
    np.testing.assert_allclose(H @ np.ones(5), 0.0, atol=1e-14)


# ---------------------------------------------------------------------------
# Descent and rates (App. A)
# ---------------------------------------------------------------------------

def _kl(p, q):
    return float(np.sum(p * np.log(p / q) - p + q))


def test_sinkhorn_one_step_descent():
    """Lemma sinkhorn-descent: f(v+) - f(v) <= -KL(b||c(v)) - KL(c(v+)||b),
    with D_phi*(0, xi) = KL(b||c) and D_phi*(xi, 0) = KL(c||b) for c = b + xi."""
    C, a, b = _problem(61, 40, 35)
    eps = 0.01
    v = np.zeros(35)
    st = O.sstep(C, eps, a, b, v)
    for _ in range(60):
        c = np.exp(v + st["ell"])
        vp = st["S"]
        stp = O.sstep(C, eps, a, b, vp)
        cp = np.exp(vp + stp["ell"])
        lhs = stp["fval"] - st["fval"]
        rhs = -_kl(b, c) - _kl(cp, b)
        assert lhs <= rhs + 1e-13 * max(1.0, abs(st["fval"]))
        v, st = vp, stp


def test_sinkhorn_sublinear_rate():
    """Thm 3.9 of the cited dual relative smoothness result with L = 1 (App. A):
    KL(c_k || b) <= (f(v_0) - f*)/k for every k >= 1."""
    C, a, b = _problem(62, 30, 30)
    eps = 0.005
    out = O.solve(C, a, b, eps, tol=1e-300, max_iter=300, method=O.SINKHORN, trace=True, trace_x=True)
    best = O.solve(C, a, b, eps, tol=1e-12, max_iter=500000, method=O.SINKHORN, trace=True)
    fstar = best["trace_fval"][-1]
    f0 = out["trace_fval"][0]
    for k in range(1, 301):
        v = out["trace_x"][k]
        c = np.exp(v + O.sstep(C, eps, a, b, v)["ell"])
        assert _kl(c, b) <= (f0 - fstar) / k + 1e-13


def test_acc_faster_rate_than_sinkhorn():
    """Theorem thm:homotopy: Acc needs O(tau^-1/2) iterations to accuracy tau,
    Sinkhorn O(tau^-1) in the sublinear regime.  Fitted on tau = 1e-2 .. 1e-5:
    the Acc exponent is clearly smaller than Sinkhorn's."""
    r = _rng(63)
    n = m = 60
    X, Y = r.uniform(size=(n, 2)), r.uniform(size=(m, 2))
    C = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    C /= C.max()
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    eps = 1e-3
    taus = np.array([1e-2, 1e-3, 1e-4, 1e-5])
    its = {}
    for method in (O.SINKHORN, O.ACC):
        out = O.solve(C, a, b, eps, tol=taus[-1], method=method, mu0=0.1, m0=10, w_rule=O.W_Y_CONTINUOUS,
                      trace=True, max_iter=200000)
        te = out["trace_err"]
        its[method] = np.array([np.argmax(te < t) for t in taus])
    sk = np.polyfit(np.log(taus), np.log(its[O.SINKHORN]), 1)[0]
    ac = np.polyfit(np.log(taus), np.log(np.maximum(its[O.ACC], 1)), 1)[0]
    assert its[O.ACC][-1] < its[O.SINKHORN][-1]
    assert ac > sk + 0.15  # slopes are negative: Acc's is flatter


# ---------------------------------------------------------------------------
# Envelope-theorem gradients
# ---------------------------------------------------------------------------

def _eot_value(C, a, b, eps):
    out = O.solve(C, a, b, eps, tol=1e-13, method=O.ACC, mu0=0.1, m0=10, w_rule=O.W_Y_CONTINUOUS,
                  max_iter=200000)
    return O.evaluate(C, eps, a, b, out["f"], out["g"])["dual"], out


def test_grad_cost_is_plan():
    """dEOT/dC_ij = P_ij, by central differences on single entries."""
    C, a, b = _problem(71, 6, 5)
    eps = 0.1
    v0, out = _eot_value(C, a, b, eps)
    P = _plan(C, eps, out["f"], out["g"])
    h = 1e-5
    for (i, j) in [(0, 0), (2, 3), (5, 4), (3, 1)]:
        E = np.zeros_like(C)
        E[i, j] = h
        fd = (_eot_value(C + E, a, b, eps)[0] - _eot_value(C - E, a, b, eps)[0]) / (2 * h)
        assert abs(fd - P[i, j]) <= 1e-7


@pytest.mark.parametrize("kind", [0, 1])
def test_grad_points_finite_differences(kind):
    """dEOT/dX, dEOT/dY (envelope theorem) vs central differences, h = 1e-4."""
    r = _rng(72 + kind)
    n, m, d = 7, 6, 3
    X, Y = r.normal(size=(n, d)), r.normal(size=(m, d))
    if kind == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    a, b = r.dirichlet(np.ones(n)), r.dirichlet(np.ones(m))
    scale, eps = 2.0 * d, 0.05

    def val(Xv, Yv):
        return _eot_value(O.cost_points(kind, Xv, Yv, scale), a, b, eps)

    v0, out = val(X, Y)
    dX, dY = O.grad_points(kind, X, Y, scale, eps, out["f"], out["g"])
    h = 1e-4
    for (i, k) in [(0, 0), (3, 2), (6, 1)]:
        E = np.zeros_like(X)
        E[i, k] = h
        fd = (val(X + E, Y)[0] - val(X - E, Y)[0]) / (2 * h)
        assert abs(fd - dX[i, k]) <= 1e-6 * max(1.0, abs(fd))
    for (j, k) in [(0, 1), (5, 0)]:
        E = np.zeros_like(Y)
        E[j, k] = h
        fd = (val(X, Y + E)[0] - val(X, Y - E)[0]) / (2 * h)
        assert abs(fd - dY[j, k]) <= 1e-6 * max(1.0, abs(fd))


def test_grad_marginals_finite_differences():
    """dEOT/da along mass-preserving directions equals <f, da> (envelope theorem);
    for raw (un-normalized) marginals the gradient is (f - <f,a>)/sum(a)."""
    C, a, b = _problem(73, 6, 5)
    a_raw, b_raw = a * 3.0, b * 0.5
    eps = 0.1
    v0, out = _eot_value(C, a, b, eps)
    da, db = O.grad_marginals(out["f"], out["g"], a_raw, b_raw)
    h = 1e-6
    for i in (0, 4):
        E = np.zeros(6)
        E[i] = h
        vp = _eot_value(C, (a_raw + E) / (a_raw + E).sum(), b, eps)[0]
        vm = _eot_value(C, (a_raw - E) / (a_raw - E).sum(), b, eps)[0]
        assert abs((vp - vm) / (2 * h) - da[i]) <= 1e-6
    for j in (1, 3):
        E = np.zeros(5)
        E[j] = h
        vp = _eot_value(C, a, (b_raw + E) / (b_raw + E).sum(), eps)[0]
        vm = _eot_value(C, a, (b_raw - E) / (b_raw - E).sum(), eps)[0]
        assert abs((vp - vm) / (2 * h) - db[j]) <= 1e-6


def test_planted_mistake_is_caught():
    """A dropped minus sign in the row solve (planted here on the CPU, in a copy
    of the step) breaks the KKT pin: the pins are not vacuous."""
    C, a, b = _problem(81, 10, 8)
    eps = 0.1
    x = np.zeros(8)
    # wrong row solve: u_i = log a_i + LSE_j(x_j - C_ij/eps)
    z = x[None, :] - C / eps
    u_bad = np.log(a) + (z.max(1) + np.log(np.exp(z - z.max(1, keepdims=True)).sum(1)))
    P = np.exp(u_bad[:, None] + x[None, :] - C / eps)
    assert np.abs(P.sum(1) - a).sum() > 1e-3
    st = O.sstep(C, eps, a, b, x)
    P = np.exp(st["u"][:, None] + x[None, :] - C / eps)
    assert np.abs(P.sum(1) - a).sum() < 1e-12


def test_stability_monitor_pins():
    """The monitor's count on plain Sinkhorn is 0 (Lemma sinkhorn-descent: f falls at
    every step); on Acc-Sinkhorn it equals the rises of the traced f(x_k) above
    1e-8 + 1e-12|f|; the restart safeguard reaches the same optimum as Sinkhorn."""
    for seed in (1, 2):
        C, a, b = _problem(seed, 60, 45)
        p = dict(a=a, b=b)
        for eps in (1e-2, 1e-3):
            sk = O.solve(C, p["a"], p["b"], eps, tol=1e-12, method=O.SINKHORN, trace=True, max_iter=200000)
            assert sk["fval_increases"] == 0
            tf = sk["trace_fval"]
            assert np.all(np.diff(tf) <= 1e-12 * np.abs(tf[1:]))  # the descent itself, in FP64
            acc = O.solve(C, p["a"], p["b"], eps, tol=1e-9, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_LITERAL,
                          trace=True, max_iter=50000)
            tf = acc["trace_fval"]
            rises = int(np.sum(tf[1:] > tf[:-1] + (1e-8 + 1e-12 * np.abs(tf[1:]))))
            assert acc["fval_increases"] == rises
            rst = O.solve(C, p["a"], p["b"], eps, tol=1e-12, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_LITERAL,
                          restart=True, max_iter=50000)
            assert rst["converged"] and rst["restarts"] == rst["fval_increases"]
            # same optimum (gauge: g centred on both sides), as Sinkhorn's
            assert np.allclose(rst["g"], sk["g"], rtol=0, atol=1e-8 * eps * 1e3)
            assert np.allclose(rst["f"], sk["f"], rtol=0, atol=1e-8 * eps * 1e3)


# ---------------------------------------------------------------------------
# The checker itself: evaluate, plan, evaluate_points and the cost builders
# ---------------------------------------------------------------------------

def _constructed(seed, n, m, eps):
    """A cost whose plan at chosen, non-optimal potentials (f, g) is a known matrix P0.

    eq:P-from-dual gives P_ij = exp((f_i + g_j - C_ij)/eps); choosing
    C_ij = f_i + g_j - eps log P0_ij makes the plan at (f, g) equal P0, so its
    marginals, mass and <C,P> follow from P0 by plain sums, with no exponential.
    P0's row and column sums straddle a and b (mixed-sign residuals) and its
    mass is not 1, so a dropped absolute value, a swapped marginal or a wrong
    exponent sign changes the result.
    """
    r = _rng(seed)
    P0 = r.uniform(0.2, 1.8, size=(n, m)) / (n * m) * 1.3
    a = r.dirichlet(np.ones(n))
    b = r.dirichlet(np.ones(m))
    f = r.normal(0.0, 0.3, n)
    g = r.normal(0.0, 0.3, m)
    C = f[:, None] + g[None, :] - eps * np.log(P0)
    return C, a, b, f, g, P0


@pytest.mark.parametrize("seed,n,m,eps", [(201, 9, 6, 0.7), (202, 5, 13, 0.05), (203, 31, 17, 2.0)])
def test_evaluate_on_constructed_plan(seed, n, m, eps):
    """oracle evaluate/plan at potentials that are not optimal, against P0's own sums."""
    C, a, b, f, g, P0 = _constructed(seed, n, m, eps)
    rs, cs = P0.sum(1), P0.sum(0)
    assert np.any(rs > a) and np.any(rs < a) and np.any(cs > b) and np.any(cs < b)
    ev = O.evaluate(C, eps, a, b, f, g)
    assert ev["row_err"] == pytest.approx(np.abs(rs - a).sum(), rel=1e-12)
    assert ev["col_err"] == pytest.approx(np.abs(cs - b).sum(), rel=1e-12)
    assert ev["err"] == pytest.approx(ev["row_err"] + ev["col_err"], rel=1e-15)
    assert ev["mass"] == pytest.approx(P0.sum(), rel=1e-12)
    assert abs(ev["mass"] - 1.0) > 0.05
    assert ev["cost"] == pytest.approx((C * P0).sum(), rel=1e-11, abs=1e-13)
    assert ev["dual"] == pytest.approx(f @ a + g @ b - eps * P0.sum(), rel=1e-11, abs=1e-13)
    np.testing.assert_allclose(O.plan(C, eps, f, g), P0, rtol=1e-12)
    np.testing.assert_allclose(O.plan(C, eps, f, g, row0=2, rows=3), P0[2:5], rtol=1e-12)


def test_evaluate_at_the_optimum_of_a_separable_cost():
    """Separable cost C_ij = alpha_i + beta_j: the optimal potentials are known in
    closed form, f_i = alpha_i + eps log a_i + c and g_j = beta_j + eps log b_j - c
    (eq:P-from-dual with P = a b^T), so both marginal errors are 0 and the mass is 1."""
    r = _rng(204)
    n, m, eps = 8, 11, 0.3
    al, be = r.uniform(0, 1, n), r.uniform(0, 1, m)
    a, b = r.dirichlet(np.ones(n)), r.dirichlet(np.ones(m))
    C = al[:, None] + be[None, :]
    f = al + eps * np.log(a) + 0.37
    g = be + eps * np.log(b) - 0.37
    ev = O.evaluate(C, eps, a, b, f, g)
    assert ev["row_err"] < 1e-14 and ev["col_err"] < 1e-14
    assert ev["mass"] == pytest.approx(1.0, abs=1e-14)
    ab = np.outer(a, b)
    assert ev["dual"] == pytest.approx(al @ a + be @ b + eps * np.sum(ab * (np.log(ab) - 1.0)), abs=1e-13)


@pytest.mark.parametrize("kind", [0, 1])
def test_cost_points_against_scipy(kind):
    """Sec. 5 costs against scipy's pairwise distances (a separate library routine)."""
    from scipy.spatial.distance import cdist
    r = _rng(205 + kind)
    X, Y = r.normal(size=(23, 7)), r.normal(size=(19, 7))
    if kind == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        ref = cdist(X, Y, "cosine") / 3.0  # 1 - x.y/(|x||y|) with unit rows
    else:
        ref = cdist(X, Y, "sqeuclidean") / 3.0
    np.testing.assert_allclose(O.cost_points(kind, X, Y, 3.0), ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", [0, 1])
def test_evaluate_points_against_stored_cost(kind):
    """evaluate_points forms each entry itself; on scipy's stored cost, evaluate
    (pinned above by construction) must give the same five values."""
    from scipy.spatial.distance import cdist
    r = _rng(207 + kind)
    n, m, d, s, eps = 37, 29, 5, 2.5, 0.08
    X, Y = r.uniform(size=(n, d)), r.uniform(size=(m, d))
    if kind == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        C = cdist(X, Y, "cosine") / s
    else:
        C = cdist(X, Y, "sqeuclidean") / s
    a, b = r.dirichlet(np.ones(n)), r.dirichlet(np.ones(m))
    f, g = r.normal(0, 0.02, n), r.normal(0, 0.02, m)
    ep = O.evaluate_points(kind, X, Y, s, eps, a, b, f, g)
    ev = O.evaluate(C, eps, a, b, f, g)
    for k in ("row_err", "col_err", "dual", "cost", "mass"):
        assert ep[k] == pytest.approx(ev[k], rel=1e-11, abs=1e-14), k
    # and at an optimum: both errors vanish on the solved problem
    out = O.solve(C, a, b, eps, tol=1e-12, method=O.SINKHORN, max_iter=100000)
    ep = O.evaluate_points(kind, X, Y, s, eps, a, b, out["f"], out["g"])
    assert ep["err"] < 1e-11
