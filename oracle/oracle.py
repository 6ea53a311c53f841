"""FP64 CPU oracle for EOT by Sinkhorn and Acc-Sinkhorn (ctypes shim + numpy forms).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this module or
the C file it loads (``accsk_oracle.c``); only the tests, the smoke check and
the CPU-baseline leg of the benchmark do.

Contents
--------
* ``solve`` / ``sstep`` / ``evaluate`` / ``evaluate_points`` / ``plan`` / cost
  builders / point-cloud gradients: thin wrappers around the plain C oracle
  (FP64 throughout).
* ``scheme_xy``: a second, independent form of the accelerated iteration written
  with the explicit auxiliary sequence y of eq:scheme (Sec. 4) and the mirror
  map grad phi*(xi) = log(1 + xi./b) of Sec. 3, in numpy, for small problems.
  Algorithm A2MD is obtained from it by w = alpha*y with alpha = sqrt(2 mu);
  the two must produce the same iterates.
* ``grad_f_fd`` helpers used by the tests that pin grad f = c_P - b (eq:grad-f).

Parity pins: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_pins.py`` against closed forms (separable cost, 2x2 plan,
Acc recurrence on a separable cost), an exact LP, invariances, descent and
rate inequalities from App. A, and finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "accsk_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

SINKHORN = 0
ACC = 1
W_LITERAL = 0
W_Y_CONTINUOUS = 1

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (portable x86-64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_sstep.argtypes = [_d, _i64, _i64, ctypes.c_double, _d, _d, _d, _d, _d, _d, _d, _d]
        lib.oracle_sstep.restype = None
        lib.oracle_solve.argtypes = [ctypes.c_int, _d, _i64, _i64, ctypes.c_double, _d, _d,
                                     ctypes.c_double, _i64, ctypes.c_double, _i64, ctypes.c_int,
                                     _d, _d, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _d,
                                     _d, _d, _d]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_solve_ex.argtypes = [ctypes.c_int, _d, _i64, _i64, ctypes.c_double, _d, _d,
                                        ctypes.c_double, _i64, ctypes.c_double, _i64, ctypes.c_int, ctypes.c_int,
                                        _d, _d, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _d,
                                        _d, _d, _d, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        lib.oracle_solve_ex.restype = ctypes.c_int
        lib.oracle_solve_mon.argtypes = lib.oracle_solve_ex.argtypes + [ctypes.POINTER(_i64), _d]
        lib.oracle_solve_mon.restype = ctypes.c_int
        lib.oracle_cond_metric.argtypes = [_d, _d, _i64, _d, _d]
        lib.oracle_cond_metric.restype = None
        lib.oracle_eval.argtypes = [_d, _i64, _i64, ctypes.c_double, _d, _d, _d, _d, _d, _d, _d, _d, _d]
        lib.oracle_eval.restype = None
        lib.oracle_eval_points.argtypes = [ctypes.c_int, _d, _d, _i64, _i64, _i64, ctypes.c_double,
                                           ctypes.c_double, _d, _d, _d, _d, _d, _d, _d, _d, _d]
        lib.oracle_eval_points.restype = None
        lib.oracle_plan.argtypes = [_d, _i64, _i64, ctypes.c_double, _d, _d, _i64, _i64, _d]
        lib.oracle_plan.restype = None
        lib.oracle_cost_sqeuclid.argtypes = [_d, _d, _i64, _i64, _i64, ctypes.c_double, _d]
        lib.oracle_cost_sqeuclid.restype = None
        lib.oracle_cost_cosine.argtypes = [_d, _d, _i64, _i64, _i64, ctypes.c_double, _d]
        lib.oracle_cost_cosine.restype = None
        lib.oracle_grad_points.argtypes = [ctypes.c_int, _d, _d, _i64, _i64, _i64, ctypes.c_double,
                                           ctypes.c_double, _d, _d, _d, _d]
        lib.oracle_grad_points.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
        return lib


def _p(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def normalize(a):
    """Marginals are scaled to unit mass, as eq:Fc requires (1'a = 1'b = 1)."""
    a = _f64(a)
    return a / a.sum()


def sstep(C, eps, a, b, x):
    """One normalized Sinkhorn step at x.  Returns dict(u, ell, S, err, fval)."""
    C = _f64(C)
    n, m = C.shape
    a, b, x = _f64(a), _f64(b), _f64(x)
    u = np.empty(n)
    ell = np.empty(m)
    S = np.empty(m)
    err = ctypes.c_double()
    fval = ctypes.c_double()
    _load().oracle_sstep(_p(C), n, m, float(eps), _p(a), _p(b), _p(x), _p(u), _p(ell), _p(S),
                         ctypes.byref(err), ctypes.byref(fval))
    return dict(u=u, ell=ell, S=S, err=err.value, fval=fval.value)


def solve(C, a, b, eps, tol=1e-6, max_iter=100000, method=ACC, mu0=0.5, m0=1,
          w_rule=W_LITERAL, trace=False, trace_x=False, normalize_marginals=True, restart=False,
          conditions=False):
    """Solve EOT(C, a, b, eps) with plain Sinkhorn or Acc-Sinkhorn (FP64).

    Returns a dict with f, g (potentials in cost units, g centred), iters, steps,
    err, converged and, if asked, per-iteration traces of err, f(x) and x.
    conditions=True (Acc) adds the boundedness monitor (App. B, Theorem
    thm:condition-boundedness): cond_counts = [violations of condition 1, of
    condition 2, rises of the shifted Lyapunov function] and trace_cond, per It
    the row (lhs1, rhs1, lhs2, rhs2, E).
    """
    C = _f64(C)
    n, m = C.shape
    if normalize_marginals:
        a, b = normalize(a), normalize(b)
    else:
        a, b = _f64(a), _f64(b)
    f = np.empty(n)
    g = np.empty(m)
    it = _i64()
    st = _i64()
    err = ctypes.c_double()
    te = np.empty(max_iter + 1) if trace else None
    tf = np.empty(max_iter + 1) if trace else None
    tx = np.empty((max_iter + 1, m)) if trace_x else None
    null = ctypes.cast(None, _d)
    ninc, nrst = _i64(), _i64()
    cc = (_i64 * 3)(-1, -1, -1)
    tc = np.full((max_iter + 1, 5), np.nan) if conditions else None
    conv = _load().oracle_solve_mon(int(method), _p(C), n, m, float(eps), _p(a), _p(b), float(tol),
                                    int(max_iter), float(mu0), int(m0), int(w_rule), int(bool(restart)), _p(f),
                                    _p(g), ctypes.byref(it), ctypes.byref(st), ctypes.byref(err),
                                    _p(te) if trace else null, _p(tf) if trace else null,
                                    _p(tx) if trace_x else null, ctypes.byref(ninc), ctypes.byref(nrst),
                                    cc if conditions else ctypes.cast(None, ctypes.POINTER(_i64)),
                                    _p(tc) if conditions else null)
    out = dict(f=f, g=g, iters=it.value, steps=st.value, err=err.value, converged=bool(conv),
               a=a, b=b, fval_increases=ninc.value, restarts=nrst.value)
    if conditions:
        out["cond_counts"] = [cc[0], cc[1], cc[2]]
        out["trace_cond"] = tc[: it.value + 1].copy()
    if trace:
        out["trace_err"] = te[: it.value + 1].copy()
        out["trace_fval"] = tf[: it.value + 1].copy()
    if trace_x:
        out["trace_x"] = tx[: it.value + 1].copy()
    return out


def cond_metric(c, b):
    """Monitor metric for column sums c: (D diagonal of eq:D, per-column terms of D_phi*(0, c - b))."""
    c, b = _f64(c), _f64(b)
    D = np.empty(len(c))
    K = np.empty(len(c))
    _load().oracle_cond_metric(_p(c), _p(b), len(c), _p(D), _p(K))
    return D, K


def evaluate(C, eps, a, b, f, g):
    """FP64 evaluation of (f, g): row/col L1 errors, EOT dual value, <C,P>, sum P."""
    C = _f64(C)
    n, m = C.shape
    a, b, f, g = _f64(a), _f64(b), _f64(f), _f64(g)
    vals = [ctypes.c_double() for _ in range(5)]
    _load().oracle_eval(_p(C), n, m, float(eps), _p(a), _p(b), _p(f), _p(g),
                        *[ctypes.byref(v) for v in vals])
    re, ce, dual, cost, mass = (v.value for v in vals)
    return dict(row_err=re, col_err=ce, err=re + ce, dual=dual, cost=cost, mass=mass)


def evaluate_points(kind, X, Y, scale, eps, a, b, f, g):
    """``evaluate`` on the point-cloud cost (kind 0 squared Euclidean, 1 cosine,
    divided by ``scale``), each entry formed in FP64 when used, nothing n x m stored."""
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    a, b, f, g = _f64(a), _f64(b), _f64(f), _f64(g)
    vals = [ctypes.c_double() for _ in range(5)]
    _load().oracle_eval_points(int(kind), _p(X), _p(Y), n, m, d, float(scale), float(eps), _p(a), _p(b), _p(f),
                               _p(g), *[ctypes.byref(v) for v in vals])
    re, ce, dual, cost, mass = (v.value for v in vals)
    return dict(row_err=re, col_err=ce, err=re + ce, dual=dual, cost=cost, mass=mass)


def plan(C, eps, f, g, row0=0, rows=None):
    C = _f64(C)
    n, m = C.shape
    rows = n - row0 if rows is None else rows
    P = np.empty((rows, m))
    _load().oracle_plan(_p(C), n, m, float(eps), _p(_f64(f)), _p(_f64(g)), int(row0), int(rows), _p(P))
    return P


def cost_sqeuclid(X, Y, scale=1.0):
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    C = np.empty((n, m))
    _load().oracle_cost_sqeuclid(_p(X), _p(Y), n, m, d, float(scale), _p(C))
    return C


def cost_cosine(X, Y, scale=1.0):
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    C = np.empty((n, m))
    _load().oracle_cost_cosine(_p(X), _p(Y), n, m, d, float(scale), _p(C))
    return C


def cost_points(kind, X, Y, scale):
    return cost_sqeuclid(X, Y, scale) if kind == 0 else cost_cosine(X, Y, scale)


def grad_points(kind, X, Y, scale, eps, f, g):
    """Envelope-theorem gradients of the EOT value w.r.t. X and Y (FP64)."""
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    dX = np.empty((n, d))
    dY = np.empty((m, d))
    _load().oracle_grad_points(int(kind), _p(X), _p(Y), n, m, d, float(scale), float(eps),
                               _p(_f64(f)), _p(_f64(g)), _p(dX), _p(dY))
    return dX, dY


def grad_marginals(f, g, a_raw, b_raw):
    """Gradient of the EOT value w.r.t. raw (un-normalized) marginals.

    The solver uses a/sum(a); by the envelope theorem dL/da_hat = f (defined up
    to a constant, eq:Fc), so dL/da_raw = (f - <f, a_hat>)/sum(a_raw).
    """
    a_raw, b_raw = _f64(a_raw), _f64(b_raw)
    ah, bh = a_raw / a_raw.sum(), b_raw / b_raw.sum()
    f, g = _f64(f), _f64(g)
    return (f - f @ ah) / a_raw.sum(), (g - g @ bh) / b_raw.sum()


# ---------------------------------------------------------------------------
# Second form of the accelerated scheme (numpy, small problems only)
# ---------------------------------------------------------------------------

def _lse(z, axis):
    mx = np.max(z, axis=axis, keepdims=True)
    return np.squeeze(mx, axis=axis) + np.log(np.sum(np.exp(z - mx), axis=axis))


def mirror_step_p(C, eps, a, b, x):
    """p(x) = P_Nperp grad phi*(P_Nperp grad f(x)), grad phi*(xi) = log(1 + xi./b).

    Built from the mirror-descent reading of Sec. 3 (eq:md-general and
    eq:normalized-sinkhorn), not from the log-domain form the C oracle uses:
    grad f = c_P(u(x), x) - b with u(x) the exact row solve (eq:grad-f).
    """
    Ct = np.asarray(C, dtype=np.float64) / eps
    u = np.log(a) - _lse(x[None, :] - Ct, axis=1)
    P = np.exp(u[:, None] + x[None, :] - Ct)
    xi = P.sum(axis=0) - b
    xi = xi - xi.mean()
    p = np.log1p(xi / b)
    return p - p.mean()


def scheme_xy(C, eps, a, b, mu, iters):
    """Iterate eq:scheme with explicit (x, y) at fixed mu for ``iters`` steps.

    (x_{k+1} - x_k)/alpha = y_k - x_{k+1} - p(x_k)/alpha
    (y_{k+1} - y_k)/alpha = x_{k+1} - y_{k+1} - p(x_{k+1})/mu
    solved for x_{k+1} and y_{k+1}, with alpha = sqrt(2 mu), x_0 = y_0 = 0.
    Returns the array of x iterates (iters+1, m).
    """
    a, b = normalize(a), normalize(b)
    m = len(b)
    alpha = np.sqrt(2.0 * mu)
    x = np.zeros(m)
    y = np.zeros(m)
    xs = [x.copy()]
    px = mirror_step_p(C, eps, a, b, x)
    for _ in range(iters):
        x = (x - px + alpha * y) / (1.0 + alpha)
        px = mirror_step_p(C, eps, a, b, x)
        y = (y + alpha * x - (alpha / mu) * px) / (1.0 + alpha)
        xs.append(x.copy())
    return np.array(xs)
