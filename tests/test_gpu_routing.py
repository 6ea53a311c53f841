"""Which solver takes a problem, and the limits of each (GPU).

* A batch of more than 64 problems puts every problem that fits one workgroup
  on one workgroup; the launch reserves on-chip memory for the largest single
  problem, so tall-narrow and short-wide problems share it (4096 x 64 next to
  64 x 1024 and 2600 x 1024).
* A problem that does not fit one workgroup's on-chip memory (4096 x 1024) is
  solved by a group of workgroups.
* A batch whose groups would need more on-chip memory than a workgroup has
  (256 problems of 600 x 8192) is split into launches that fit.
* A single problem whose row blocks cannot fit on chip at one block per CU
  (900000 x 1025, 3.7 GB of cost) goes to the tiled solver.
* A launch of 16 problems with 1500 to 1911 columns runs the wave-rows kernel
  with 32 columns per lane.

Bars as in the batch parity tests (FP64 marginal error <= tol, stopping
iterate against the oracle's trace, dual value); identical problems in one
call give identical bits.  At 900000 x 1025 the oracle checks sampled rows one
by one; the column marginals are summed in FP64 with plain PyTorch.
"""
import numpy as np
import pytest

from oracle import oracle as O

from _stopcheck import check_stop
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _oracle_check(p, f, g, r, tol=1e-6):
    from paper_2605_30267_amd import accsk
    C = p["C32"].astype(np.float64)
    an, bn = p["a"] / p["a"].sum(), p["b"] / p["b"].sum()
    ev = O.evaluate(C, p["eps"], an, bn, f, g)
    print("  ", C.shape, "It", r["iters"], "err", ev["err"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1, r
    assert ev["err"] <= tol
    assert abs(r["eot_value"] - ev["dual"]) <= 2e-7 * p["eps"] + 1e-12 * abs(ev["dual"])
    dp = accsk.default_params()
    check_stop(C, an, bn, p["eps"], tol, O.ACC, r["iters"], dp.mu0, dp.m0, dp.w_rule)


def test_large_batch_one_workgroup_mixed_shapes(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    kinds = [W.random_dense(501, 4096, 64, eps=1e-2), W.random_dense(502, 64, 1024, eps=1e-2),
             W.random_dense(503, 2600, 1024, eps=3e-2)]
    dev = [(_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
            _dev(torch, p["b"], torch.float64), p["eps"]) for p in kinds]
    batch = [dev[k % 3] for k in range(66)]
    print("case 66-problem batch of 4096x64, 64x1024, 2600x1024", flush=True)
    outs, res, st = accsk.solve_batch(batch)
    torch.cuda.synchronize()
    assert st == accsk.OK
    for k in range(3):
        _oracle_check(kinds[k], outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy(), res[k])
    for k in range(3, 66):
        assert torch.equal(outs[k][0], outs[k % 3][0]) and torch.equal(outs[k][1], outs[k % 3][1])
        assert res[k]["iters"] == res[k % 3]["iters"]


def test_beyond_one_workgroup(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(504, 4096, 1024, eps=1e-2, a_kind="dirichlet")
    print("case 4096x1024 in a batch and alone", flush=True)
    dev = (_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64),
           p["eps"])
    outs, res, st = accsk.solve_batch([dev] * 70)  # also above 64 problems: still a group of workgroups each
    torch.cuda.synchronize()
    assert st == accsk.OK
    _oracle_check(p, outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy(), res[0])
    f, g, r = accsk.solve_dense(*dev)
    torch.cuda.synchronize()
    _oracle_check(p, f.cpu().numpy(), g.cpu().numpy(), r)


def test_batch_split_into_fitting_launches(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(505, 600, 8192, eps=2e-2, a_kind="dirichlet")
    dev = (_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64), _dev(torch, p["b"], torch.float64),
           p["eps"])
    print("case 256 x (600x8192)", flush=True)
    outs, res, st = accsk.solve_batch([dev] * 256)
    torch.cuda.synchronize()
    assert st == accsk.OK
    _oracle_check(p, outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy(), res[0])
    for k in range(1, 256):
        assert torch.equal(outs[k][0], outs[0][0]) and torch.equal(outs[k][1], outs[0][1])


def test_tall_single_problem_tiled_fallback(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    n, m, eps, tol = 900000, 1025, 5e-2, 1e-6
    gen = torch.Generator(device="cuda")
    gen.manual_seed(506)
    print("case 900000x1025 single", flush=True)
    C = torch.rand(n, m, device="cuda", dtype=torch.float32, generator=gen)
    a = torch.rand(n, device="cuda", dtype=torch.float64, generator=gen) + 0.5
    b = torch.rand(m, device="cuda", dtype=torch.float64, generator=gen) + 0.5
    f, g, r = accsk.solve_dense(C, a, b, eps, tol=tol)
    torch.cuda.synchronize()
    print("  It", r["iters"], "err", r["marginal_err"], "kernel ms", r["kernel_ms"], flush=True)
    assert r["status"] == 0 and r["converged"] == 1, r
    an = (a / a.sum()).cpu().numpy()
    bn = (b / b.sum()).cpu().numpy()
    fh, gh = f.cpu().numpy(), g.cpu().numpy()
    # sampled rows, one by one in FP64: the returned f solves its rows exactly
    rng = np.random.default_rng(0)
    rows = rng.choice(n, 32, replace=False)
    Cr = C[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
    for k, i in enumerate(rows):
        ri = np.exp((fh[i] + gh - Cr[k]) / eps).sum()
        assert abs(ri - an[i]) <= 1e-6 * an[i]
    # column marginals over all rows, FP64
    col = torch.zeros(m, dtype=torch.float64, device="cuda")
    fd, gd = f.view(-1, 1), g.view(1, -1)
    for r0 in range(0, n, 100000):
        col += torch.exp((fd[r0:r0 + 100000] + gd - C[r0:r0 + 100000].double()) / eps).sum(0)
    err = float(torch.abs(col - torch.as_tensor(bn, device="cuda")).sum())
    print("  FP64 column error", err, flush=True)
    assert err <= tol


@pytest.mark.parametrize("widths", [(1500, 1637, 1774, 1911), (1500, 1600, 1800, 2048)])
def test_wave_rows_wide_batch(torch_gpu, widths):
    """m in (1024, 2048] in a launch of 16 problems: the wave-rows kernel with 32 columns per lane,
    with 4-byte loads (some m not a multiple of 4) and with 16-byte loads (two waves per SIMD)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    kinds = [W.random_dense(510 + k, 300, w, eps=1e-2, a_kind="dirichlet") for k, w in enumerate(widths)]
    dev = [(_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
            _dev(torch, p["b"], torch.float64), p["eps"]) for p in kinds]
    batch = [dev[k % 4] for k in range(16)]
    print("case 16-problem batch, m =", widths, flush=True)
    outs, res, st = accsk.solve_batch(batch)
    torch.cuda.synchronize()
    assert st == accsk.OK
    for k in range(2):
        _oracle_check(kinds[k], outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy(), res[k])
    for k in range(4, 16):
        assert torch.equal(outs[k][0], outs[k % 4][0]) and torch.equal(outs[k][1], outs[k % 4][1])


def test_workspace_bound(torch_gpu):
    """The workspace bound covers the cooperative launch's column partials and grows with the problem."""
    from paper_2605_30267_amd import accsk
    w1 = accsk.workspace_bytes(8192, 8192)
    # one cooperative launch keeps one FP32 and two FP64 column partials per workgroup and column
    assert w1 >= 256 * 8192 * (4 + 16)
    assert accsk.workspace_bytes(16384, 8192) > w1 and accsk.workspace_bytes(8192, 8192, 64) >= w1
    assert accsk.workspace_bytes(100, 20000) >= 512 * 20000 * (4 + 16)  # tiled: two workgroups per CU
    assert accsk.workspace_bytes(64, 64, 1024) >= 1024 * 2 * 64


@pytest.mark.parametrize("n,m", [(100000, 1), (40000, 3), (1, 8192), (2, 5000), (70000, 200)])
def test_extreme_aspect_ratios(torch_gpu, n, m):
    """Very tall and very wide problems on the cooperative solver (most lanes' columns masked, or a
    single row for the whole launch)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(520 + m, n, m, eps=1e-2, a_kind="dirichlet")
    print("case aspect", n, m, flush=True)
    f, g, r = accsk.solve_dense(_dev(torch, p["C32"], torch.float32), _dev(torch, p["a"], torch.float64),
                                _dev(torch, p["b"], torch.float64), 1e-2)
    torch.cuda.synchronize()
    _oracle_check(p, f.cpu().numpy(), g.cpu().numpy(), r)
