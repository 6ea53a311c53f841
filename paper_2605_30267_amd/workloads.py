"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (point clouds, marginals, dense costs, request
streams).  It holds none of the solver's arithmetic and is shared by the tests,
the benchmark and the smoke check; both the GPU library and the FP64 oracle are
fed from it.  Every generator uses ``numpy.random.default_rng(seed)`` and draws
in the order written in its docstring.

Workloads (the paper's own data -- two photographs, fastText vectors and the
MUSE dictionary of Sec. 5 -- are not available, so these stand in for them):

* ``small_uniform``     n = m = 256, points U[0,1]^2, sq-Euclidean / max,
                        a, b ~ U(0.5, 1.5) normalized, eps = 1e-2.
* ``gmm_dense``         n = m = 8192, 4-component 2-D Gaussian mixtures
                        (means U[0,1]^2, sigma 0.1), sq-Euclidean / max as FP32,
                        a, b ~ Dirichlet(1); eps in {1e-2, 1e-3, 1e-4}.
* ``color_points``      n = m = 32768 RGB points from 8-cluster mixtures
                        (centres U[0,1]^3, proportions Dirichlet(1_8), sigma 0.05,
                        clipped to [0,1]^3); weights proportional to the point's
                        cluster share; eps = 1e-3 (colour-transfer stand-in).
* ``word_requests``     a stream of solves with n, m ~ U{8..256}, unit-norm
                        N(0, I_300) embeddings, uniform marginals, eps from
                        {1e-2, 3e-3, 1e-3}, Poisson arrival times (word-alignment
                        stand-in).
* ``gaussian_batch``    B problems with X, Y ~ N(0, I_64), n = m = 2048,
                        uniform marginals, eps = 5e-3.
* ``paper_synthetic``   Sec. 5 "Synthetic Datasets": a, b, C with entries
                        U[0,1], a and b normalized to unit sum, C scaled to sum 1.
* ``color_table``       n = 1000 RGB points per side as in ``color_points``,
                        uniform marginals, explicit sq-Euclidean / max cost: the
                        size and marginals of Sec. 5's colour-transfer table.
* ``word_table``        n = 500 unit vectors in d = 300 and a hidden permutation:
                        y_pi(i) is x_i plus Gaussian noise, renormalized; uniform
                        marginals, cosine cost: the size of Sec. 5's
                        word-alignment table, with a known ground truth for the
                        top-1 / top-5 readout.
* ``outlier_columns``   tests only: U[0, 0.5] costs with a few columns raised
                        by 0.5, so that at small eps they get almost no mass at
                        the start.
"""
from __future__ import annotations

import numpy as np


def _sq_dist_over_max(X, Y, chunk=1024):
    """Dense ||x_i - y_j||^2 divided by its maximum, computed in FP64 by rows."""
    n, m = X.shape[0], Y.shape[0]
    C = np.empty((n, m), dtype=np.float64)
    for i0 in range(0, n, chunk):
        Xi = X[i0:i0 + chunk]
        D = Xi[:, None, :] - Y[None, :, :]
        C[i0:i0 + chunk] = np.einsum("ijk,ijk->ij", D, D)
    return C / C.max()


def small_uniform(seed=1, n=256, m=256):
    """X ~ U[0,1]^2 (drawn first), Y ~ U[0,1]^2, a ~ U(0.5,1.5), b ~ U(0.5,1.5).

    Returns dict(C32 [n,m] float32, a, b [float64, unit sum], eps=1e-2).
    """
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 2))
    Y = rng.uniform(0.0, 1.0, size=(m, 2))
    a = rng.uniform(0.5, 1.5, size=n)
    b = rng.uniform(0.5, 1.5, size=m)
    C = _sq_dist_over_max(X, Y).astype(np.float32)
    return dict(C32=C, a=a / a.sum(), b=b / b.sum(), eps=1e-2, X=X, Y=Y)


def _gmm2d(rng, count, k=4, sigma=0.1):
    means = rng.uniform(0.0, 1.0, size=(k, 2))
    comp = rng.integers(0, k, size=count)
    return means[comp] + sigma * rng.standard_normal(size=(count, 2))


def gmm_dense(seed=2, n=8192, m=8192, eps=1e-2):
    """Draw order: X mixture (means, components, noise), Y mixture, a ~ Dir(1_n), b ~ Dir(1_m).

    Returns dict(C32 float32 [n,m] row-major, a, b float64 unit sum, eps).
    """
    rng = np.random.default_rng(seed)
    X = _gmm2d(rng, n)
    Y = _gmm2d(rng, m)
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    C = _sq_dist_over_max(X, Y).astype(np.float32)
    return dict(C32=C, a=a, b=b, eps=eps, X=X, Y=Y)


def _rgb_clusters(rng, count, k=8, sigma=0.05):
    centres = rng.uniform(0.0, 1.0, size=(k, 3))
    props = rng.dirichlet(np.ones(k))
    comp = rng.choice(k, size=count, p=props)
    pts = np.clip(centres[comp] + sigma * rng.standard_normal(size=(count, 3)), 0.0, 1.0)
    share = np.bincount(comp, minlength=k) / count
    w = share[comp]
    return pts, w / w.sum()


def color_points(seed=3, n=32768, m=32768, eps=1e-3):
    """Draw order: X (centres, proportions, labels, noise), then Y the same way.

    Returns float32 X [n,3], Y [m,3] and float64 weights a, b (unit sum).
    """
    rng = np.random.default_rng(seed)
    X, a = _rgb_clusters(rng, n)
    Y, b = _rgb_clusters(rng, m)
    return dict(X=X.astype(np.float32), Y=Y.astype(np.float32), a=a, b=b, eps=eps)


def unit_rows(rng, count, d):
    Z = rng.standard_normal(size=(count, d))
    return Z / np.linalg.norm(Z, axis=1, keepdims=True)


def word_requests(seed=4, count=4000, d=300, rate=None, eps_set=(1e-2, 3e-3, 1e-3),
                  nmin=8, nmax=256):
    """Per request, in order: n, m ~ U{nmin..nmax}, eps index, X [n,d], Y [m,d].

    Arrival gaps ~ Exp(rate) drawn afterwards from ``default_rng(seed * 10)``
    (rate None -> all arrive at t = 0).  Marginals are uniform.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        m = int(rng.integers(nmin, nmax + 1))
        eps = float(eps_set[int(rng.integers(0, len(eps_set)))])
        X = unit_rows(rng, n, d).astype(np.float32)
        Y = unit_rows(rng, m, d).astype(np.float32)
        reqs.append(dict(X=X, Y=Y, a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), eps=eps))
    arr = np.zeros(count) if rate is None else poisson_arrivals(count, rate, seed * 10)
    for r, t in zip(reqs, arr):
        r["arrival"] = float(t)
    return reqs


def poisson_arrivals(count, rate, seed=40):
    """Arrival instants (seconds from 0) of a Poisson process: cumulative Exp(rate) gaps."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


def gaussian_batch(seed=5, batch=64, n=2048, m=2048, d=64, eps=5e-3):
    """Draw order: X [batch,n,d] then Y [batch,m,d], i.i.d. N(0,1), float32."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(size=(batch, n, d)).astype(np.float32)
    Y = rng.standard_normal(size=(batch, m, d)).astype(np.float32)
    a = np.full((batch, n), 1.0 / n)
    b = np.full((batch, m), 1.0 / m)
    return dict(X=X, Y=Y, a=a, b=b, eps=eps, scale=2.0 * d)


def paper_synthetic(seed=6, n=100, m=50, eps=1e-8):
    """Sec. 5 synthetic: a, b, C entries U[0,1]; a, b to unit sum; C to unit total."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=n)
    b = rng.uniform(0.0, 1.0, size=m)
    C = rng.uniform(0.0, 1.0, size=(n, m))
    return dict(C=C / C.sum(), a=a / a.sum(), b=b / b.sum(), eps=eps)


def color_table(seed=7, n=1000):
    """Draw order: X clusters then Y clusters (as ``color_points``); a = b = 1/n.

    Returns float32 X, Y [n,3], C32 = ||x - y||^2 / max over the FP32 points
    (FP64, rounded to FP32), a, b.
    """
    rng = np.random.default_rng(seed)
    X, _ = _rgb_clusters(rng, n)
    Y, _ = _rgb_clusters(rng, n)
    X32, Y32 = X.astype(np.float32), Y.astype(np.float32)
    C = _sq_dist_over_max(X32.astype(np.float64), Y32.astype(np.float64)).astype(np.float32)
    return dict(X=X32, Y=Y32, C32=C, a=np.full(n, 1.0 / n), b=np.full(n, 1.0 / n))


WORD_NOISE = 4.5  # nearest-neighbour top-1 of the stand-in is about 3/4


def word_table(seed=8, n=500, d=300, noise=WORD_NOISE):
    """Draw order: X [n,d] ~ N(0,I) rows, a permutation pi of n, Z [n,d] ~ N(0,I).

    x_i = X_i/|X_i|; y_pi(i) = u/|u| with u = x_i + noise * Z_i / sqrt(d).
    Returns float32 X, Y (unit rows), truth = pi (row i's partner is column
    pi[i]), a = b = 1/n.  The cost is the cosine distance 1 - <x, y> divided
    by its maximum (see ``accsk.cost_max_points``).
    """
    rng = np.random.default_rng(seed)
    X = unit_rows(rng, n, d)
    perm = rng.permutation(n)
    Z = rng.standard_normal(size=(n, d)) / np.sqrt(d)
    U = X + noise * Z
    Y = np.empty_like(X)
    Y[perm] = U / np.linalg.norm(U, axis=1, keepdims=True)
    return dict(X=X.astype(np.float32), Y=Y.astype(np.float32), truth=perm, a=np.full(n, 1.0 / n),
                b=np.full(n, 1.0 / n))


def random_dense(seed, n, m, eps=1e-2, a_kind="uniform"):
    """Small generic dense problem for tests: C ~ U[0,1] as float32, positive marginals."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, size=(n, m)).astype(np.float32)
    if a_kind == "dirichlet":
        a = rng.dirichlet(np.ones(n))
        b = rng.dirichlet(np.ones(m))
    else:
        a = rng.uniform(0.5, 1.5, size=n)
        b = rng.uniform(0.5, 1.5, size=m)
        a, b = a / a.sum(), b / b.sum()
    return dict(C32=C, a=a, b=b, eps=eps)


def outlier_columns(seed, n, m, eps=1e-4, frac=0.02, lift=0.5):
    """Test problem with columns no row reaches at the start: C ~ U[0, 0.5] as
    float32, then a random `frac` of the columns raised by `lift`; marginals
    U(0.5, 1.5) normalized.  Draw order: C, the raised columns, a, b.  At small
    eps those columns receive almost no mass in the first steps (the degenerate
    start the solvers' exact column pass handles)."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 0.5, size=(n, m))
    cols = rng.choice(m, max(1, int(frac * m)), replace=False)
    C[:, cols] += lift
    a = rng.uniform(0.5, 1.5, size=n)
    b = rng.uniform(0.5, 1.5, size=m)
    return dict(C32=C.astype(np.float32), a=a / a.sum(), b=b / b.sum(), eps=eps, cols=np.sort(cols))
