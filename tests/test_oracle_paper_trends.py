"""Pins of the FP64 oracle against the iteration behaviour Sec. 5 reports.

The paper's data (photographs, word vectors) are not available, so these run on
the seeded stand-ins of ``workloads`` at reduced size (n = 200) and check the
trends its experiments report, not its exact counts:

* synthetic problems (Sec. 5, "Synthetic Datasets", n = 100, m = 50,
  eps = 1e-8): Acc-Sinkhorn reaches a given marginal error in more than ten
  times fewer iterations than Sinkhorn at moderate accuracy;
* colour transfer (Sec. 5 colour table, tol = 2/n): both methods need a
  handful of iterations at eps = 1 and 0.1, and the Sinkhorn / Acc-Sinkhorn
  iteration ratio grows as eps falls, past 10 at eps = 1e-4;
* word alignment (Sec. 5 word table, tol = 0.02/n): the ratio is large at every
  eps <= 1e-2.

A broken extrapolation or homotopy schedule in the oracle loses the
acceleration and fails these; the closed forms and exact checks of
``test_oracle_pins.py`` cover the arithmetic itself.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_30267_amd import workloads as W

MU0, M0 = 0.25, 5  # the library's calibrated homotopy start (also the oracle's setting in every GPU test)


def _solve(C, a, b, eps, tol, method, **kw):
    extra = dict(mu0=MU0, m0=M0, w_rule=O.W_Y_CONTINUOUS) if method == O.ACC else {}
    return O.solve(C, a, b, eps, tol=tol, method=method, max_iter=10 ** 6, **extra, **kw)


def _first_below(trace, tol):
    hit = np.nonzero(np.asarray(trace) < tol)[0]
    return int(hit[0]) if hit.size else None


def test_synthetic_e1_acc_ten_times_fewer_iterations():
    """n = 100, m = 50, eps = 1e-8, entries U[0,1] (Sec. 5 synthetic datasets)."""
    p = W.paper_synthetic(n=100, m=50, eps=1e-8)
    acc = _solve(p["C"], p["a"], p["b"], p["eps"], 1e-4, O.ACC, trace=True)["trace_err"]
    sk = _solve(p["C"], p["a"], p["b"], p["eps"], 1e-4, O.SINKHORN, trace=True)["trace_err"]
    for tol in (1e-3, 1e-4):
        ka, ks = _first_below(acc, tol), _first_below(sk, tol)
        print("tol", tol, "Acc It", ka, "Sinkhorn It", ks, flush=True)
        assert ka is not None and ks is not None
        assert ks >= 10 * ka


def test_colour_table_trend():
    c = W.color_table(n=200)
    C = c["C32"].astype(np.float64)
    tol = 2.0 / 200
    ratios = []
    for eps in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        ka = _solve(C, c["a"], c["b"], eps, tol, O.ACC)["iters"]
        ks = _solve(C, c["a"], c["b"], eps, tol, O.SINKHORN)["iters"]
        print("eps", eps, "Acc It", ka, "Sinkhorn It", ks, flush=True)
        if eps >= 1e-1:
            assert ka <= 6 and ks <= 6
        else:
            ratios.append(ks / ka)
    assert ratios[0] < ratios[1] < ratios[2]
    assert ratios[2] >= 10


def test_word_table_trend():
    w = W.word_table(n=200)
    C = O.cost_points(1, w["X"], w["Y"], 1.0)
    C = C / C.max()
    tol = 0.02 / 200
    for eps in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        ka = _solve(C, w["a"], w["b"], eps, tol, O.ACC)["iters"]
        ks = _solve(C, w["a"], w["b"], eps, tol, O.SINKHORN)["iters"]
        print("eps", eps, "Acc It", ka, "Sinkhorn It", ks, flush=True)
        if eps >= 1e-1:
            assert ka <= 6 and ks <= 6
        else:
            assert ks >= 5 * ka
