"""GPU parity of the point-cloud paths: cost construction, point-cloud solves
(single and batched), and the envelope-theorem backward.

Costs (Sec. 5: squared Euclidean, cosine) are checked against the FP64
oracle element by element:
  * split 0 (FP64 dot products, one rounding to FP32): |dC| <= 2^-24 |C| + 1e-14;
  * split 2 / 3 (BF16 pieces on the matrix cores, FP32 accumulation per 32-wide
    chunk): |dC_ij| <= 2^-14 (resp. 2^-20) * B_ij with B_ij = (|x_i|^2 + |y_j|^2)/s
    for squared Euclidean and |x_i||y_j|/s for cosine.  A wrong matrix-core
    operand or result layout gives errors of order B itself.
Solves are judged on FP64 quantities computed by the oracle on its own cost
(rounded to FP32 as the library stores it).  Gradients are compared at the
oracle's potentials (FP32 exponentials of FP64 arguments, FP64 sums, FP32
output: relative 2e-6 of the largest entry).
"""
import numpy as np
import pytest

from oracle import oracle as O

from _stopcheck import STOP, check_stop
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _clouds(seed, n, m, d, kind):
    rng = np.random.default_rng(seed)
    if kind == 1:
        X = W.unit_rows(rng, n, d).astype(np.float32)
        Y = W.unit_rows(rng, m, d).astype(np.float32)
    else:
        X = rng.standard_normal(size=(n, d)).astype(np.float32)
        Y = (rng.standard_normal(size=(m, d)) + 0.5).astype(np.float32)
    return X, Y


def _bound(X, Y, kind, s):
    X, Y = X.astype(np.float64), Y.astype(np.float64)
    nx, ny = np.linalg.norm(X, axis=1), np.linalg.norm(Y, axis=1)
    if kind == 0:
        return (nx[:, None] ** 2 + ny[None, :] ** 2) / s
    return nx[:, None] * ny[None, :] / s


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n,m,d", [(70, 133, 3), (33, 65, 64), (129, 47, 300), (1, 1, 1), (17, 5, 512)])
def test_cost_fp64(torch_gpu, kind, n, m, d):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(11 + n, n, m, d, kind)
    s = 2.0 * d if kind == 0 else 1.0
    C = accsk.cost_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), kind=kind,
                          cost_scale=s, split=0).cpu().numpy().astype(np.float64)
    ref = O.cost_points(kind, X, Y, s)
    err = np.abs(C - ref)
    print("kind", kind, (n, m, d), "max |dC|", err.max(), flush=True)
    assert np.all(err <= 2.0 ** -24 * np.abs(ref) + 1e-14)


@pytest.mark.parametrize("split,rel", [(2, 2.0 ** -14), (3, 2.0 ** -20)])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n,m,d", [(70, 133, 3), (64, 96, 64), (45, 77, 300), (1, 2, 1), (33, 31, 100)])
def test_cost_mfma(torch_gpu, split, rel, kind, n, m, d):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(23 + n, n, m, d, kind)
    s = 2.0 * d if kind == 0 else 1.0
    C = accsk.cost_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), kind=kind,
                          cost_scale=s, split=split).cpu().numpy().astype(np.float64)
    ref = O.cost_points(kind, X, Y, s)
    B = _bound(X, Y, kind, s)
    q = np.abs(C - ref) / B
    print("split", split, "kind", kind, (n, m, d), "max |dC|/B", q.max(), "(bound %.3g)" % rel, flush=True)
    assert np.all(q <= rel)


def test_cost_leading_dim_and_errors(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(5, 20, 30, 8, 0)
    Xd, Yd = _dev(torch, X, torch.float32), _dev(torch, Y, torch.float32)
    big = torch.full((20, 37), -7.0, dtype=torch.float32, device="cuda")
    accsk.cost_points(Xd, Yd, split=0, out=big[:, :30])
    torch.cuda.synchronize()
    host = big.cpu().numpy()
    assert np.all(host[:, 30:] == -7.0)  # padding columns untouched
    assert np.allclose(host[:, :30], O.cost_points(0, X, Y, 1.0), rtol=1e-6, atol=0)
    lib = accsk._points_lib()
    stream = accsk._stream_ptr()
    out = torch.empty((20, 30), dtype=torch.float32, device="cuda")
    p = accsk._ptr
    assert lib.accsk_cost_points(p(Xd), p(Yd), 20, 30, 8, 0, 1.0, 1, p(out), 30, stream) == accsk.INVALID_ARG
    assert lib.accsk_cost_points(p(Xd), p(Yd), 20, 30, 8, 2, 1.0, 0, p(out), 30, stream) == accsk.INVALID_ARG
    assert lib.accsk_cost_points(p(Xd), p(Yd), 20, 30, 8, 0, 0.0, 0, p(out), 30, stream) == accsk.INVALID_ARG
    assert lib.accsk_cost_points(p(Xd), p(Yd), 20, 30, 8, 0, 1.0, 0, p(out), 29, stream) == accsk.SHAPE
    assert lib.accsk_cost_points(p(Xd), p(Yd), 20, 30, 513, 0, 1.0, 0, p(out), 30, stream) == accsk.SHAPE
    assert lib.accsk_cost_points(p(Xd), p(Yd), 0, 30, 8, 0, 1.0, 0, p(out), 30, stream) == accsk.SHAPE


def _check_solution(X, Y, a, b, kind, s, eps, f, g, r, tol, method=1, stop=True):
    C32 = O.cost_points(kind, X, Y, s).astype(np.float32).astype(np.float64)
    an, bn = a / a.sum(), b / b.sum()
    ev = O.evaluate(C32, eps, an, bn, f, g)
    print("shape", C32.shape, "eps", eps, "It", r["iters"], "err", ev["err"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1, r
    # the library's cost may differ from fl32(oracle cost) by one FP32 rounding in rare entries
    assert ev["err"] <= tol * 1.001
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * eps + 1e-12 * abs(ev["dual"])
    if stop:
        dp = __import__("paper_2605_30267_amd.accsk", fromlist=["x"]).default_params()
        check_stop(C32, an, bn, eps, tol, O.ACC if method == 1 else O.SINKHORN, r["iters"], dp.mu0, dp.m0,
                   dp.w_rule)
    return ev


@pytest.mark.parametrize("kind,n,m,d,eps", [(0, 300, 257, 3, 1e-2), (1, 60, 90, 300, 3e-3),
                                            (0, 1, 7, 2, 1e-2), (0, 1500, 1100, 8, 2e-2)])
def test_solve_points(torch_gpu, kind, n, m, d, eps):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(31 + n, n, m, d, kind)
    rng = np.random.default_rng(n + m)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d) if kind == 0 else 1.0
    f, g, res = accsk.solve_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                   _dev(torch, a, torch.float64), _dev(torch, b, torch.float64), eps, kind=kind,
                                   cost_scale=s, split=0, tol=1e-6)
    torch.cuda.synchronize()
    _check_solution(X, Y, a, b, kind, s, eps, f.cpu().numpy(), g.cpu().numpy(), res[0], 1e-6)


def test_solve_points_batched_equals_alone(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    B, n, m, d, eps = 3, 200, 150, 16, 1e-2
    p = W.gaussian_batch(seed=9, batch=B, n=n, m=m, d=d, eps=eps)
    Xd, Yd = _dev(torch, p["X"], torch.float32), _dev(torch, p["Y"], torch.float32)
    ad, bd = _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64)
    f, g, res = accsk.solve_points(Xd, Yd, ad, bd, eps, cost_scale=p["scale"])
    torch.cuda.synchronize()
    for k in range(B):
        fk, gk, rk = accsk.solve_points(Xd[k], Yd[k], ad[k], bd[k], eps, cost_scale=p["scale"])
        torch.cuda.synchronize()
        assert torch.equal(fk, f[k]) and torch.equal(gk, g[k])
        assert rk[0]["iters"] == res[k]["iters"]
        _check_solution(p["X"][k], p["Y"][k], p["a"][k], p["b"][k], 0, p["scale"], eps, f[k].cpu().numpy(),
                        g[k].cpu().numpy(), res[k], 1e-6)


@pytest.mark.parametrize("split", [0, 3])
def test_solve_points_gaussian_full(torch_gpu, split):
    """Two problems of the batched Gaussian workload at full size (2048 x 2048, d = 64, eps 5e-3)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.gaussian_batch(seed=5, batch=2, n=2048, m=2048, d=64, eps=5e-3)
    f, g, res = accsk.solve_points(_dev(torch, p["X"], torch.float32), _dev(torch, p["Y"], torch.float32),
                                   _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64),
                                   p["eps"], cost_scale=p["scale"], split=split)
    torch.cuda.synchronize()
    for k in range(2):
        r = res[k]
        C = O.cost_points(0, p["X"][k], p["Y"][k], p["scale"])
        if split == 0:
            _check_solution(p["X"][k], p["Y"][k], p["a"][k], p["b"][k], 0, p["scale"], p["eps"],
                            f[k].cpu().numpy(), g[k].cpu().numpy(), r, 1e-6, stop=False)
        else:
            # the solve ran on the split-3 cost: its marginals on the exact cost are off by at most
            # the cost error times 1/eps in the exponent (relative 2^-20 * B / eps per entry)
            ev = O.evaluate(C, p["eps"], p["a"][k], p["b"][k], f[k].cpu().numpy(), g[k].cpu().numpy())
            bound = 2.0 ** -20 * _bound(p["X"][k], p["Y"][k], 0, p["scale"]).max() / p["eps"]
            print("split 3 exact-cost err", ev["err"], "bound", 2 * bound + 1e-6, flush=True)
            assert r["converged"] == 1 and ev["err"] <= 2 * bound + 1e-6


@pytest.mark.parametrize("kind,n,m,d,eps", [(0, 40, 33, 5, 5e-2), (1, 24, 70, 300, 1e-2),
                                            (0, 1, 1, 1, 1e-1), (0, 37, 130, 448, 2e-2), (1, 90, 17, 64, 1e-2)])
def test_backward_points(torch_gpu, kind, n, m, d, eps):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(41 + n, n, m, d, kind)
    rng = np.random.default_rng(3 * n + m)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d) if kind == 0 else 1.0
    C = O.cost_points(kind, X, Y, s)
    o = O.solve(C, a, b, eps, tol=1e-11, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    fo, go = o["f"], o["g"]
    gsc = 1.75
    dX, dY, da, db = accsk.backward_points(
        _dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), _dev(torch, a, torch.float64),
        _dev(torch, b, torch.float64), _dev(torch, fo, torch.float64), _dev(torch, go, torch.float64), eps,
        kind=kind, cost_scale=s, grad_scale=torch.tensor([gsc], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    rX, rY = O.grad_points(kind, X, Y, s, eps, fo, go)
    ra, rb = O.grad_marginals(fo, go, a, b)
    for got, ref, name in ((dX, rX, "dX"), (dY, rY, "dY")):
        got = got.cpu().numpy().astype(np.float64) / gsc
        e = np.abs(got - ref).max()
        print(name, "max err", e, "scale", np.abs(ref).max(), flush=True)
        assert e <= 2e-6 * np.abs(ref).max() + 1e-300
    # FP64: the weighted mean <f, a>/sum(a) is rounded, so the absolute scale is |f|/sum(a)
    assert np.allclose(da.cpu().numpy() / gsc, ra, rtol=1e-12, atol=1e-14 * np.abs(fo).max() / a.sum())
    assert np.allclose(db.cpu().numpy() / gsc, rb, rtol=1e-12, atol=1e-14 * np.abs(go).max() / b.sum())


def test_backward_errors(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    lib = accsk._points_lib()
    p = accsk._ptr
    X = torch.zeros((4, 449), dtype=torch.float32, device="cuda")
    f = torch.zeros(4, dtype=torch.float64, device="cuda")
    out = torch.empty_like(X)
    st = lib.accsk_backward_points(p(X), p(X), 1, 4, 4, 449, 0, 1.0, 0.1, None, None, p(f), p(f), None, p(out),
                                   p(out), None, None, accsk._stream_ptr())
    assert st == accsk.SHAPE
    st = lib.accsk_backward_points(p(X), p(X), 1, 4, 4, 8, 0, 1.0, 0.0, None, None, p(f), p(f), None, p(out),
                                   p(out), None, None, accsk._stream_ptr())
    assert st == accsk.INVALID_ARG


def test_eot_loss_autograd(torch_gpu):
    """torch.autograd through the library: weighted sum of two problems' EOT values."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    B, n, m, d, eps = 2, 50, 40, 6, 5e-2
    p = W.gaussian_batch(seed=12, batch=B, n=n, m=m, d=d, eps=eps)
    rng = np.random.default_rng(1)
    a, b = rng.uniform(0.5, 1.5, (B, n)), rng.uniform(0.5, 1.5, (B, m))
    Xd = _dev(torch, p["X"], torch.float32).requires_grad_(True)
    Yd = _dev(torch, p["Y"], torch.float32).requires_grad_(True)
    ad = _dev(torch, a, torch.float64).requires_grad_(True)
    bd = _dev(torch, b, torch.float64).requires_grad_(True)
    vals = accsk.eot_loss(Xd, Yd, ad, bd, eps, cost_scale=p["scale"], tol=1e-9)
    wts = torch.tensor([2.0, -0.5], dtype=torch.float64, device="cuda")
    (vals * wts).sum().backward()
    torch.cuda.synchronize()
    for k in range(B):
        C = O.cost_points(0, p["X"][k], p["Y"][k], p["scale"])
        o = O.solve(C, a[k], b[k], eps, tol=1e-11, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
        ev = O.evaluate(C, eps, a[k] / a[k].sum(), b[k] / b[k].sum(), o["f"], o["g"])
        assert abs(vals[k].item() - ev["dual"]) <= 1e-6 * eps
        rX, rY = O.grad_points(0, p["X"][k], p["Y"][k], p["scale"], eps, o["f"], o["g"])
        ra, rb = O.grad_marginals(o["f"], o["g"], a[k], b[k])
        w = wts[k].item()
        # potentials converge to tol 1e-9 (not the oracle's 1e-12): gradients agree to ~1e-6 relative
        for got, ref in ((Xd.grad[k], rX), (Yd.grad[k], rY), (ad.grad[k], ra), (bd.grad[k], rb)):
            got = got.detach().cpu().numpy().astype(np.float64) / w
            assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("kind,n,m,d", [(0, 70, 133, 3), (1, 40, 90, 300), (0, 1, 1, 1)])
def test_plan_points(torch_gpu, kind, n, m, d):
    """P rows on demand from the points at the oracle's potentials (row range with an offset)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(51 + n, n, m, d, kind)
    rng = np.random.default_rng(n)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d) if kind == 0 else 1.0
    eps = 2e-2
    C = O.cost_points(kind, X, Y, s)
    o = O.solve(C, a, b, eps, tol=1e-10, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    row0 = n // 3
    rows = n - row0
    P = accsk.plan_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                          _dev(torch, o["f"], torch.float64), _dev(torch, o["g"], torch.float64), eps, kind=kind,
                          cost_scale=s, row0=row0, rows=rows)
    torch.cuda.synchronize()
    ref = O.plan(C, eps, o["f"], o["g"], row0, rows)
    got = P.cpu().numpy().astype(np.float64)
    big = ref > 1e-30
    assert np.all(np.abs(got[big] - ref[big]) <= 2.0 ** -23 * ref[big])
    assert abs(got.sum() - ref.sum()) <= 1e-6 * ref.sum()


@pytest.mark.parametrize("kind,n,m,d", [(0, 70, 133, 3), (1, 40, 190, 300), (0, 33, 1, 2)])
def test_barycentric_points(torch_gpu, kind, n, m, d):
    """T_i = sum_j P_ij y_j / sum_j P_ij (colour-transfer map) at the oracle's potentials."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(61 + n, n, m, d, kind)
    rng = np.random.default_rng(m)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d) if kind == 0 else 1.0
    eps = 2e-2
    C = O.cost_points(kind, X, Y, s)
    o = O.solve(C, a, b, eps, tol=1e-10, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    T = accsk.barycentric_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                 _dev(torch, o["f"], torch.float64), _dev(torch, o["g"], torch.float64), eps,
                                 kind=kind, cost_scale=s)
    torch.cuda.synchronize()
    P = O.plan(C, eps, o["f"], o["g"])
    ref = (P @ Y.astype(np.float64)) / P.sum(axis=1, keepdims=True)
    got = T.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-6 * max(1.0, np.abs(Y).max())


@pytest.mark.parametrize("k", [1, 5, 8])
@pytest.mark.parametrize("kind,n,m,d", [(0, 70, 133, 3), (1, 50, 300, 300), (0, 9, 4, 2)])
def test_topk_points(torch_gpu, k, kind, n, m, d):
    """Row top-k of P decided on g_j - C_ij in FP64; where the order differs from the
    oracle's it must be a tie to FP64 rounding of the cost."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    X, Y = _clouds(71 + n + k, n, m, d, kind)
    rng = np.random.default_rng(n + k)
    a, b = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    s = float(d) if kind == 0 else 1.0
    eps = 1e-2
    C = O.cost_points(kind, X, Y, s)
    o = O.solve(C, a, b, eps, tol=1e-9, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    idx, val = accsk.topk_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32),
                                 _dev(torch, o["f"], torch.float64), _dev(torch, o["g"], torch.float64), eps, k=k,
                                 kind=kind, cost_scale=s)
    torch.cuda.synchronize()
    idx, val = idx.cpu().numpy(), val.cpu().numpy()
    score = o["g"][None, :] - C
    kk = min(k, m)
    for i in range(n):
        order = np.lexsort((np.arange(m), -score[i]))[:kk]
        got = idx[i, :kk]
        assert len(set(got.tolist())) == kk and np.all(got >= 0)
        # same scores in the same order (ties resolved either way only within FP64 rounding)
        assert np.allclose(score[i, got], score[i, order], rtol=0, atol=1e-12 * (1 + np.abs(score[i]).max()))
        np.testing.assert_allclose(val[i, :kk], np.exp((o["f"][i] + score[i, got]) / eps), rtol=1e-12)
        if kk < k:
            assert np.all(idx[i, kk:] == -1)


@pytest.mark.parametrize("kind,split,B,n,m,d", [(0, 3, 5, 37, 70, 45), (1, 2, 3, 130, 17, 300), (0, 2, 2, 64, 64, 64),
                                                (1, 3, 4, 1, 5, 1)])
def test_cost_points_batched_equals_single(torch_gpu, kind, split, B, n, m, d):
    """One launch for a batch of problems gives each problem's cost bit for bit as its own call
    (same pieces, products and sums); ragged n, m (not multiples of 16 or 64) and d (not of 32)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    rng = np.random.default_rng(B * 100 + n)
    X = rng.standard_normal((B, n, d)).astype(np.float32)
    Y = rng.standard_normal((B, m, d)).astype(np.float32)
    if kind == 1:
        X /= np.linalg.norm(X, axis=2, keepdims=True)
        Y /= np.linalg.norm(Y, axis=2, keepdims=True)
    s = 2.0 * d if kind == 0 else 1.0
    print("case batched cost", kind, split, B, n, m, d, flush=True)
    Cb = accsk.cost_points(_dev(torch, X, torch.float32), _dev(torch, Y, torch.float32), kind=kind, cost_scale=s,
                           split=split)
    for k in range(B):
        Ck = accsk.cost_points(_dev(torch, X[k], torch.float32), _dev(torch, Y[k], torch.float32), kind=kind,
                               cost_scale=s, split=split)
        assert torch.equal(Cb[k], Ck), k
    # and the split bound against the exact FP64 cost (as for single problems)
    Cx = O.cost_points(kind, X[0], Y[0], s)
    B0 = (np.sum(X[0].astype(np.float64) ** 2, 1)[:, None] + np.sum(Y[0].astype(np.float64) ** 2, 1)[None, :]) / s \
        if kind == 0 else np.outer(np.linalg.norm(X[0], axis=1), np.linalg.norm(Y[0], axis=1)) / s
    rel = 2.0 ** -20 if split == 3 else 2.0 ** -14
    assert np.all(np.abs(Cb[0].cpu().numpy().astype(np.float64) - Cx) <= rel * B0 + 2.0 ** -24 * np.abs(Cx) + 1e-30)
