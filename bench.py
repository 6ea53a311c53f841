"""Benchmark: dense explicit-cost Acc-Sinkhorn solves on one MI355X.

Workload: n = m = 8192 dense FP32 squared-Euclidean cost (max-normalized) of two
4-component 2-D Gaussian mixtures, Dirichlet(1) marginals, tol 1e-6 on the L1
marginal error; eps = 1e-3 for the headline value (1e-2 and 1e-4 reported as
context).  One "step" of this benchmark is one complete solve (set-up, all
iterations, final FP64 cost pass) with the inputs already resident in HBM.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--context", type=int, default=1, help="also time Sinkhorn and other eps (1/0)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--with-copy", action="store_true", help="run the copy calibration first, in the same process")
    ap.add_argument("--color", type=int, default=1, help="also time the colour-transfer on-the-fly solve (1/0)")
    ap.add_argument("--serving", type=int, default=1, help="also run the serving stream (1/0)")
    ap.add_argument("--diff", type=int, default=1, help="also time the differentiable batched loss (1/0)")
    ap.add_argument("--small-batch", type=int, default=1, help="also time a batch of 1024 small problems (1/0)")
    ap.add_argument("--fly-mfma", type=int, default=1,
                    help="also time the on-the-fly matrix-core solve at 32768^2, d = 64 (1/0)")
    ap.add_argument("--paper", type=int, default=1,
                    help="also run the Sec. 5 experiment shapes: synthetic, colour and word tables (1/0)")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--serve-split", type=int, default=3, help="cost split of the served requests (0, 2, 3)")
    ap.add_argument("--serve-budget-mib", type=float, default=16.0,
                    help="serving arena (HBM budget for the requests' costs), MiB")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_name(m):
    """Instantiation of the persistent solve kernel the library picks for m columns."""
    if m <= 256:
        return "dense_solve<256,1,1,WK=1> (wave rows)"
    if m <= 512:
        return "dense_solve<256,1,1,WK=2> (wave rows)"
    if m <= 1024:
        return "dense_solve<256,1,1,WK=4> (wave rows)"
    if m <= 2048:
        return "dense_solve<512,1,4>"
    if m <= 4096:
        return "dense_solve<1024,1,2>"
    return "dense_solve<1024,2,1>"


def copy_calibration(gib=1.0):
    """Plain device copy of a known size, for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 3}))


def traffic_from_profile():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    src = os.path.join(ROOT, "paper_2605_30267_amd", "csrc", "accsk_dense.hip")
    path = os.path.join(ROOT, "profiles", "dense_solve_gmm8192_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        d = json.load(fh)
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if d.get("source_sha256") != h:
        return None, None
    return d.get("hbm_bytes_per_launch"), d


# FP32 exponentials the on-the-fly (tiled) solver evaluates per cost entry and
# Sinkhorn step: one in the row sweep, one in the column sweep.
TILED_EXPS_PER_ENTRY = 2
# v_exp_f32 ceiling from the unit counts and the clock: 256 CUs x 4 SIMDs x 64 lanes,
# one exponential instruction per 8 cycles per wave (CDNA4 doubled the transcendental
# rate of CDNA3's 16), 2.4 GHz: 1.97e13 exponentials/s
EXP_PEAK = 256 * 4 * 64 / 8 * 2.4e9


def color_bench(args, dev):
    """Colour-transfer-shaped solve: n = m = 32768 RGB points, cost / exact max,
    formed on the fly in every step (never stored), eps = 1e-3, tol 1e-6."""
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    p = W.color_points(seed=3, n=32768, m=32768, eps=1e-3)
    X, Y = torch.as_tensor(p["X"], device=dev), torch.as_tensor(p["Y"], device=dev)
    a = torch.as_tensor(p["a"], dtype=torch.float64, device=dev)
    b = torch.as_tensor(p["b"], dtype=torch.float64, device=dev)
    s = accsk.cost_max_points(X, Y)
    accsk.solve_points(X, Y, a, b, p["eps"], cost_scale=s, on_the_fly=True)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    outs = [accsk.solve_points(X, Y, a, b, p["eps"], cost_scale=s, on_the_fly=True) for _ in range(reps)]
    torch.cuda.synchronize()
    rs = [o[2][0] for o in outs]
    rs_f = (outs[0][0], outs[0][1])
    dt = (time.perf_counter() - t0) / reps
    r = rs[0]
    n = m = 32768
    kms = sum(x["kernel_ms"] for x in rs) / reps
    # Minimum work per Sinkhorn step: one exponential per entry (the dense solver
    # shows that the row and column sums can share it); the bound is the FP32
    # exponential unit.  The exponentials this kernel actually evaluates per
    # entry and step are reported beside it.
    entries = float(n) * m * r["sinkhorn_steps"]
    achieved = entries / (kms * 1e-3)
    out = dict(workload="colour-transfer-shaped: n=m=32768 RGB points (8-cluster mixtures), sq-Euclidean cost "
                        "/ exact max, formed on the fly, eps=1e-3, tol=1e-6, Acc-Sinkhorn",
               solves_per_s=1.0 / dt, ms_per_solve=1e3 * dt, iters=r["iters"], sinkhorn_steps=r["sinkhorn_steps"],
               fallback_steps=r["fallback_steps"], converged=r["converged"], marginal_err=r["marginal_err"],
               kernel_ms=kms, us_per_step=1e3 * kms / r["sinkhorn_steps"],
               exps_per_entry_and_step=TILED_EXPS_PER_ENTRY,
               roofline={"bound": "alu", "achieved": achieved, "peak": EXP_PEAK, "unit": "entries/s",
                         "frac": achieved / EXP_PEAK,
                         "note": "one FP32 exponential per cost entry and Sinkhorn step (the minimum), against "
                                 "the v_exp_f32 ceiling 256 CU x 4 SIMD x 64 lanes / 8 cycles x 2.4 GHz",
                         "exp_rate": achieved * TILED_EXPS_PER_ENTRY,
                         "exp_frac": achieved * TILED_EXPS_PER_ENTRY / EXP_PEAK})
    # The same ceiling measured on this device (independent exponential chains
    # with nothing else in the loop), the exponential counterpart of the
    # measured read stream.
    exp_meas = accsk.exp_rate(reps=5)
    out["roofline"]["measured_exp_rate"] = exp_meas
    out["roofline"]["frac_of_measured"] = achieved / exp_meas
    log("colour transfer: It %d, %.1f ms/solve, %.1f us/step, frac of the exp ceiling %.3f"
        % (r["iters"], 1e3 * dt, out["us_per_step"], out["roofline"]["frac"]))
    return out, dict(X=X, Y=Y, a=a, b=b, scale=s, eps=p["eps"], res=r, f=rs_f[0], g=rs_f[1])


BF16_MFMA_PEAK = 2.5e15     # MI355X dense BF16 matrix-core peak, flop/s
FP64_PEAK = 78.6e12         # MI355X FP64 vector peak, flop/s


def timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def diff_bench(args, dev):
    """Differentiable EOT loss: 64 problems, n = m = 2048, d = 64, N(0, I) points,
    cost / (2 d), eps = 5e-3, BF16x3 matrix-core cost, forward Acc-Sinkhorn then
    the envelope-theorem backward (P recomputed tile by tile)."""
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    B, n, m, d = 64, 2048, 2048, 64
    p = W.gaussian_batch(seed=5, batch=B, n=n, m=m, d=d, eps=5e-3)
    X = torch.as_tensor(p["X"], device=dev)
    Y = torch.as_tensor(p["Y"], device=dev)
    a = torch.as_tensor(p["a"], dtype=torch.float64, device=dev)
    b = torch.as_tensor(p["b"], dtype=torch.float64, device=dev)
    s = p["scale"]

    def fwd_bwd():
        Xr = X.clone().requires_grad_(True)
        Yr = Y.clone().requires_grad_(True)
        vals = accsk.eot_loss(Xr, Yr, a, b, p["eps"], cost_scale=s, split=3)
        vals.sum().backward()
        return vals, Xr.grad

    fwd_bwd()
    t_all, (vals, gx) = timed(fwd_bwd, 2)
    t_fwd, (f, g, res) = timed(lambda: accsk.solve_points(X, Y, a, b, p["eps"], cost_scale=s, split=3), 2)
    t_bwd, _ = timed(lambda: accsk.backward_points(X, Y, a, b, f, g, p["eps"], cost_scale=s), 3)
    Cb = torch.empty((B, n, m), dtype=torch.float32, device=dev)  # the forward's 1 GiB of costs, one launch
    t_cost, _ = timed(lambda: accsk.cost_points(X, Y, cost_scale=s, split=3, out=Cb), 3)
    del Cb
    its = [r["iters"] for r in res]
    cost_flops = B * n * m * d * 2.0 * 6  # six BF16 products per split-3 cross term
    # backward, per side and entry: d FMA (cost) and d FMA (P times points), 2 flop each
    bwd_flops = 2.0 * B * n * m * (2 * d) * 2
    out = dict(workload="differentiable EOT loss: 64 problems, n=m=2048, d=64, N(0,I) points, cost/128, eps=5e-3, "
                        "BF16x3 cost, forward Acc-Sinkhorn + envelope-theorem backward",
               problems_per_s=B / t_all, ms_fwd_bwd=1e3 * t_all, ms_forward=1e3 * t_fwd, ms_backward=1e3 * t_bwd,
               mean_iters=sum(its) / B, all_converged=all(r["converged"] == 1 for r in res),
               cost_build={"ms": 1e3 * t_cost, "tflops": cost_flops / t_cost / 1e12,
                           "frac_of_bf16_peak": cost_flops / t_cost / BF16_MFMA_PEAK},
               backward={"ms": 1e3 * t_bwd, "tflops_fp64": bwd_flops / t_bwd / 1e12,
                         "frac_of_fp64_peak": bwd_flops / t_bwd / FP64_PEAK})
    log("diff loss: %.1f problems/s (fwd %.1f ms, bwd %.1f ms), cost build %.1f TFLOP/s, backward %.1f TFLOP/s"
        % (out["problems_per_s"], out["ms_forward"], out["ms_backward"], out["cost_build"]["tflops"],
           out["backward"]["tflops_fp64"]))
    dX, dY, _, _ = accsk.backward_points(X, Y, a, b, f, g, p["eps"], cost_scale=s, marginals=False)
    torch.cuda.synchronize()
    return out, dict(X=X, Y=Y, a=a, b=b, f=f, g=g, dX=dX, dY=dY, scale=s, eps=p["eps"])


def fly_mfma_bench(args, dev):
    """Cost formed on the matrix cores in every step, never stored: n = m = 32768
    N(0, I) points in d = 64, cost / (2 d), eps = 2e-2, split 3, Acc-Sinkhorn to
    tol 1e-6 (C would take 4 GiB).  Matrix-core rate: six BF16 products of the
    16 x 16 x 64 cross term per tile, two sweeps per Sinkhorn step."""
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    n = m = 32768
    d = 64
    p = W.gaussian_batch(seed=9, batch=1, n=n, m=m, d=d, eps=2e-2)
    X = torch.as_tensor(p["X"][0], device=dev)
    Y = torch.as_tensor(p["Y"][0], device=dev)
    a = torch.as_tensor(p["a"][0], dtype=torch.float64, device=dev)
    b = torch.as_tensor(p["b"][0], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, g, res = accsk.solve_points(X, Y, a, b, p["eps"], cost_scale=p["scale"], split=3, on_the_fly=True,
                                   max_iter=3000, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = res[0]
    steps = r["sinkhorn_steps"] + r["fallback_steps"]  # an exact column fallback is one more sweep pair
    flops_per_step = 2.0 * (float(n) * m * 64 * 2 * 6)
    rate = flops_per_step * steps / (r["kernel_ms"] * 1e-3)
    out = dict(workload="on the fly, BF16x3 matrix-core cross term: n=m=32768, d=64, N(0,I) points, cost/128, "
                        "eps=2e-2, tol=1e-6, Acc-Sinkhorn (C never stored; 4 GiB if it were)",
               seconds=dt, kernel_ms=r["kernel_ms"], iters=r["iters"], sinkhorn_steps=r["sinkhorn_steps"],
               fallback_steps=r["fallback_steps"], converged=r["converged"], marginal_err=r["marginal_err"],
               us_per_step=1e3 * r["kernel_ms"] / r["sinkhorn_steps"],
               mfma={"tflops": rate / 1e12, "peak_tflops": BF16_MFMA_PEAK / 1e12, "frac": rate / BF16_MFMA_PEAK,
                     "note": "split-3 products (6 BF16 MFMA per 16x16x32 block of the cross term), "
                             "row and column sweep per step"})
    log("on the fly (MFMA, d=64): It %d, %.1f ms/solve, %.0f us/step, %.1f TFLOP/s = %.3f of BF16 peak"
        % (r["iters"], 1e3 * dt, out["us_per_step"], rate / 1e12, rate / BF16_MFMA_PEAK))
    return out


def small_batch_bench(args, dev):
    """1024 independent problems shaped like the 256 x 256 uniform case (eps 1e-2),
    one workgroup each, handed over as one strided batch; HBM rate of the cost
    reads (every step streams all 268 MB of costs) and exponentials per second."""
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    B = 1024
    C = torch.empty((B, 256, 256), dtype=torch.float32, device=dev)
    a = torch.empty((B, 256), dtype=torch.float64, device=dev)
    b = torch.empty((B, 256), dtype=torch.float64, device=dev)
    for k in range(B):
        q = W.small_uniform(seed=1000 + k)
        C[k].copy_(torch.as_tensor(q["C32"]))
        a[k].copy_(torch.as_tensor(q["a"]))
        b[k].copy_(torch.as_tensor(q["b"]))
    accsk.solve_batch_strided(C[:8], a[:8], b[:8], 1e-2)
    t, (f, g, res, st) = timed(lambda: accsk.solve_batch_strided(C, a, b, 1e-2, flags=accsk.FLAG_NO_COST), 2)
    steps = float(res["sinkhorn_steps"].sum())
    exps = steps * 256.0 * 256.0  # one exponential per entry and step (row and column sums share it)
    kt = float(res["kernel_ms"][0]) * 1e-3  # the launch that solved all 1024 problems
    # the 1024 costs (268 MB) exceed the 256 MB last-level cache: every step streams them from HBM
    hbm = steps * 256.0 * 256.0 * 4.0 / kt / 1e9
    out = dict(workload="1024 independent 256x256 problems (uniform points, cost/max, U(0.5,1.5) marginals), "
                        "eps=1e-2, Acc-Sinkhorn, tol 1e-6, one workgroup per problem",
               problems_per_s=1024 / t, ms=1e3 * t, kernel_ms=1e3 * kt, problems_per_s_kernel=1024 / kt,
               mean_iters=float(res["iters"].mean()),
               all_converged=bool((res["converged"] == 1).all()), exp_per_s=exps / kt,
               frac_of_exp_peak=exps / kt / EXP_PEAK,
               roofline={"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": hbm / HBM_PEAK_GBPS, "note": "one read of each cost per Sinkhorn step"})
    log("small batch: %.0f problems/s (%.0f/s in the kernel), %.0f GB/s of costs (%.2f of HBM), %.2e exp/s"
        % (out["problems_per_s"], out["problems_per_s_kernel"], hbm, hbm / HBM_PEAK_GBPS, out["exp_per_s"]))
    return out


# Iteration counts of the paper's Sec. 5 tables, (Acc-Sinkhorn, Sinkhorn) per eps,
# measured on its own photographs and word vectors: context beside the stand-ins.
PAPER_COLOUR_IT = {1.0: (3, 1), 1e-1: (5, 4), 1e-2: (18, 37), 1e-3: (46, 359), 1e-4: (239, 3507)}
PAPER_WORD_IT = {1.0: (4, 1), 1e-1: (6, 4), 1e-2: (234, 5085), 1e-3: (268, 8254), 1e-4: (667, 20320)}
PAPER_WORD_TOP = {1.0: (76.7, 94.0), 1e-1: (78.0, 94.8), 1e-2: (82.8, 95.3), 1e-3: (81.9, 95.7), 1e-4: (82.8, 94.8)}


def paper_bench(args, dev):
    """The shapes of the Sec. 5 experiments on seeded stand-ins, both methods.

    * synthetic: n = 100, m = 50 and n = m = 100, eps = 1e-8, entries U[0,1]; It and
      solve time to tol 1e-3 .. 1e-6, plus the spread of It over mu0 x m0 at 1e-6;
    * colour table: n = 1000 RGB points, uniform marginals, tol = 2/n, eps 1 .. 1e-4;
    * word table: n = 500 unit vectors (d = 300) with a planted alignment, cosine
      cost / max, tol = 0.02/n, eps 1 .. 1e-4, top-1 / top-5 accuracy of the plan.
    """
    import numpy as np
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    def solve(C, a, b, eps, tol, method, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f, g, r = accsk.solve_dense(C, a, b, eps, tol=tol, method=method, max_iter=2000000, raise_on_error=False,
                                    **kw)
        torch.cuda.synchronize()
        return f, g, dict(iters=r["iters"], converged=r["converged"], kernel_ms=round(r["kernel_ms"], 4),
                          ms=round(1e3 * (time.perf_counter() - t0), 4))

    def dev3(C, a, b):
        return (torch.as_tensor(np.ascontiguousarray(C), dtype=torch.float32, device=dev),
                torch.as_tensor(a, dtype=torch.float64, device=dev), torch.as_tensor(b, dtype=torch.float64, device=dev))

    out = {"synthetic": {}, "colour_table": {}, "word_table": {}}
    for n, m in ((100, 50), (100, 100)):
        p = W.paper_synthetic(n=n, m=m, eps=1e-8)
        C, a, b = dev3(p["C"].astype(np.float32), p["a"], p["b"])
        solve(C, a, b, 1e-8, 1e-3, accsk.ACC)
        rows = {}
        for tol in (1e-3, 1e-4, 1e-5, 1e-6):
            ra = solve(C, a, b, 1e-8, tol, accsk.ACC)[2]
            rs = solve(C, a, b, 1e-8, tol, accsk.SINKHORN)[2]
            rows["tol=%g" % tol] = dict(acc=ra, sinkhorn=rs, it_ratio=round(rs["iters"] / max(ra["iters"], 1), 2),
                                        time_ratio=round(rs["kernel_ms"] / ra["kernel_ms"], 2))
            log("paper synthetic %dx%d tol %g: Acc It %d (%.2f ms), Sinkhorn It %d (%.2f ms)"
                % (n, m, tol, ra["iters"], ra["kernel_ms"], rs["iters"], rs["kernel_ms"]))
        sweep = {}
        for mu0 in (0.5, 0.25, 0.1):
            for m0 in (2, 5, 10):
                sweep["mu0=%g,m0=%d" % (mu0, m0)] = solve(C, a, b, 1e-8, 1e-6, accsk.ACC, mu0=mu0, m0=m0)[2]["iters"]
        rows["acc_it_over_mu0_m0_at_1e-6"] = sweep
        out["synthetic"]["%dx%d" % (n, m)] = rows

    c = W.color_table(n=1000)
    C, a, b = dev3(c["C32"], c["a"], c["b"])
    for eps in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        ra = solve(C, a, b, eps, 2e-3, accsk.ACC)[2]
        rs = solve(C, a, b, eps, 2e-3, accsk.SINKHORN)[2]
        out["colour_table"]["eps=%g" % eps] = dict(acc=ra, sinkhorn=rs, paper_it=PAPER_COLOUR_IT[eps])
        log("paper colour n=1000 eps %g: Acc It %d (%.2f ms), Sinkhorn It %d (%.2f ms)"
            % (eps, ra["iters"], ra["kernel_ms"], rs["iters"], rs["kernel_ms"]))

    w = W.word_table(n=500)
    Xd = torch.as_tensor(w["X"], device=dev)
    Yd = torch.as_tensor(w["Y"], device=dev)
    ad = torch.as_tensor(w["a"], dtype=torch.float64, device=dev)
    bd = torch.as_tensor(w["b"], dtype=torch.float64, device=dev)
    s = accsk.cost_max_points(Xd, Yd, kind=accsk.COSINE)
    truth = w["truth"]
    for eps in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        row = {}
        for name, method in (("acc", accsk.ACC), ("sinkhorn", accsk.SINKHORN)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, g, res = accsk.solve_points(Xd, Yd, ad, bd, eps, kind=accsk.COSINE, cost_scale=s, tol=0.02 / 500,
                                           method=method, max_iter=2000000)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            idx, _ = accsk.topk_points(Xd, Yd, f, g, eps, k=5, kind=accsk.COSINE, cost_scale=s)
            idx = idx.cpu().numpy()
            row[name] = dict(iters=res[0]["iters"], converged=res[0]["converged"],
                             kernel_ms=round(res[0]["kernel_ms"], 4), ms=round(ms, 4),
                             top1=round(100.0 * float(np.mean(idx[:, 0] == truth)), 1),
                             top5=round(100.0 * float(np.mean([truth[i] in idx[i] for i in range(500)])), 1))
        row["paper_it"] = PAPER_WORD_IT[eps]
        row["paper_top1_top5"] = PAPER_WORD_TOP[eps]
        out["word_table"]["eps=%g" % eps] = row
        log("paper word n=500 eps %g: Acc It %d (%.2f ms) top1 %.1f top5 %.1f, Sinkhorn It %d (%.2f ms)"
            % (eps, row["acc"]["iters"], row["acc"]["kernel_ms"], row["acc"]["top1"], row["acc"]["top5"],
               row["sinkhorn"]["iters"], row["sinkhorn"]["kernel_ms"]))
    return out


def serving_bench(args, dev):
    """Word-alignment-shaped request stream through the serving loop.

    Requests: n, m ~ U{8..256}, d = 300 unit vectors, cosine cost, uniform
    marginals, eps ~ U{1e-2, 3e-3, 1e-3}, tol 1e-6, inputs resident in HBM.
    First all requests at t = 0 (saturated throughput), then Poisson arrivals
    at 0.8 x that rate; latency = completion on the host - scheduled arrival.
    The same arrival stream is replayed with plain Sinkhorn.
    """
    import numpy as np
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    count = args.serve_requests
    log("serving: generating %d requests" % count)
    reqs = W.word_requests(seed=4, count=count, d=300)
    D = []
    for r in reqs:
        n, m = len(r["a"]), len(r["b"])
        D.append((torch.as_tensor(r["X"], device=dev), torch.as_tensor(r["Y"], device=dev),
                  torch.as_tensor(r["a"], device=dev), torch.as_tensor(r["b"], device=dev), r["eps"],
                  torch.empty(n, dtype=torch.float64, device=dev), torch.empty(m, dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()
    del reqs

    def run(method, arrivals):
        with accsk.Server(hbm_budget=int(args.serve_budget_mib * (1 << 20)), method=method,
                          split=args.serve_split) as srv:
            X, Y, a, b, eps, f, g = D[0]
            srv.wait(srv.submit(X, Y, a, b, eps, kind=accsk.COSINE, f_out=f, g_out=g))  # first launch
            t0 = accsk.clock_seconds() + 1e-3
            tickets = []
            for k, (X, Y, a, b, eps, f, g) in enumerate(D):
                if arrivals is not None:
                    target = t0 + arrivals[k]
                    while accsk.clock_seconds() < target:
                        pass
                tickets.append(srv.submit(X, Y, a, b, eps, kind=accsk.COSINE, f_out=f, g_out=g))
            outs = [srv.wait(t, timeout=900.0) for t in tickets]
            workers = srv.info()["workers"]
            adm = srv.admission()
        sub = np.array([o[3][0] for o in outs])
        done = np.array([o[3][2] for o in outs])
        start = sub if arrivals is None else t0 + arrivals  # saturated: from submission
        lat = 1e3 * (done - start)
        span = done.max() - start.min()
        its = np.array([o[2]["iters"] for o in outs])
        conv = all(o[2]["converged"] == 1 for o in outs)
        nconv = sum(o[2]["converged"] != 1 for o in outs)
        return dict(solves_per_s=count / span, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()), mean_iters=float(its.mean()),
                    all_converged=conv, not_converged=int(nconv), max_iter=100000,
                    device_ms_mean=float(np.mean([o[2]["kernel_ms"] for o in outs])),
                    device_p50_ms=float(np.percentile([o[2]["kernel_ms"] for o in outs], 50)),
                    device_p99_ms=float(np.percentile([o[2]["kernel_ms"] for o in outs], 99)), workers=workers,
                    admission=adm,
                    admit_wait_p99_ms=float(np.percentile([1e3 * (o[3][1] - o[3][0]) for o in outs], 99)))

    out = {"workload": "word-alignment-shaped stream: %d requests, n,m ~ U{8..256}, d=300, cosine cost, "
                       "eps ~ U{1e-2,3e-3,1e-3}, tol 1e-6, BF16x%d cost, %.0f MiB arena"
                       % (count, args.serve_split, args.serve_budget_mib)}
    sat = run(accsk.ACC, None)
    log("serving acc saturated: %.0f solves/s, %d requests waited for arena space (peak %.1f MiB in use)"
        % (sat["solves_per_s"], sat["admission"]["space_waited"], sat["admission"]["peak_bytes_in_use"] / 2**20))
    lam = 0.8 * sat["solves_per_s"]
    arrivals = W.poisson_arrivals(count, lam, seed=40)
    acc = run(accsk.ACC, arrivals)
    log("serving acc at %.0f/s: p50 %.2f ms p99 %.2f ms (solve on the device: p50 %.2f ms, p99 %.2f ms)"
        % (lam, acc["p50_ms"], acc["p99_ms"], acc["device_p50_ms"], acc["device_p99_ms"]))
    sk_sat = run(accsk.SINKHORN, None)
    sk = run(accsk.SINKHORN, arrivals)
    log("serving sinkhorn at %.0f/s: p50 %.2f ms p99 %.2f ms (saturated %.0f/s)"
        % (lam, sk["p50_ms"], sk["p99_ms"], sk_sat["solves_per_s"]))
    out.update(arrival_rate=lam, acc_saturated=sat, acc=acc, sinkhorn_saturated=sk_sat, sinkhorn=sk)
    return out


def cpu_baseline_leg(args, p, gpu_steps, fh, gh, r_head, color_x, diff_x):
    """The FP64 oracle beside the GPU, outside every timed region.

    * Baseline: oracle Sinkhorn steps on the headline input, on all host threads
      for about args.cpu_seconds, then on one thread for a few steps, scaled by
      the GPU's steps per Acc solve.
    * Errors against the oracle: FP64 evaluation of the headline solve's (f, g)
      on its cost; of the colour-transfer solve's (f, g) on the exact point
      cost (all 32768^2 entries, formed on the fly); envelope-theorem gradients
      of two differentiable-loss problems at the GPU's potentials.
    """
    import numpy as np

    from oracle import oracle as O
    n, m = p["C32"].shape
    Cd = p["C32"].astype(np.float64)
    an, bn = O.normalize(p["a"]), O.normalize(p["b"])
    threads = O.num_threads()

    def per_step(seconds, max_steps):
        x = np.zeros(m)
        nst = 0
        c0 = time.perf_counter()
        while True:
            st = O.sstep(Cd, args.eps, an, bn, x)
            x = st["S"]
            nst += 1
            if time.perf_counter() - c0 > seconds or nst >= max_steps:
                break
        return (time.perf_counter() - c0) / nst, nst

    log("cpu baseline: oracle Sinkhorn steps on %d threads" % threads)
    t_all, n_all = per_step(args.cpu_seconds, 1 << 30)
    O.set_threads(1)
    t_one, n_one = per_step(args.cpu_seconds / 3.0, 3)
    O.set_threads(threads)
    cpu = {"value": 1.0 / (t_all * gpu_steps), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": "%d FP64 oracle Sinkhorn steps on the same %dx%d input (%.3f s/step on %d threads), scaled "
                     "by the %d steps per Acc solve of the GPU run" % (n_all, n, m, t_all, threads, round(gpu_steps)),
           "one_thread": {"value": 1.0 / (t_one * gpu_steps), "unit": "solves/s", "cores": 1,
                          "sample": "%d steps, %.3f s/step" % (n_one, t_one)}}
    log("cpu baseline: %.3f s/step on %d threads, %.3f s/step on 1" % (t_all, threads, t_one))

    ev = O.evaluate(Cd, args.eps, an, bn, fh, gh)
    err = {"headline": {"fp64_marginal_err": ev["err"], "row_err": ev["row_err"], "col_err": ev["col_err"],
                        "eot_value_gpu": r_head["eot_value"], "eot_value_oracle_at_gpu_potentials": ev["dual"],
                        "transport_cost_gpu": r_head["transport_cost"], "transport_cost_oracle": ev["cost"],
                        "tol": 1e-6, "within_tol": bool(ev["err"] <= 1e-6)}}
    log("oracle check, headline: FP64 marginal err %.3e" % ev["err"])
    if color_x is not None:
        c = color_x
        t0 = time.perf_counter()
        ec = O.evaluate_points(0, c["X"].cpu().numpy(), c["Y"].cpu().numpy(), c["scale"], c["eps"],
                               O.normalize(c["a"].cpu().numpy()), O.normalize(c["b"].cpu().numpy()),
                               c["f"].cpu().numpy(), c["g"].cpu().numpy())
        err["colour_transfer"] = {"fp64_marginal_err_exact_cost": ec["err"], "row_err": ec["row_err"],
                                  "col_err": ec["col_err"], "eot_value_gpu": c["res"]["eot_value"],
                                  "eot_value_oracle_at_gpu_potentials": ec["dual"],
                                  "entries": float(c["X"].shape[0]) * c["Y"].shape[0],
                                  "oracle_seconds": time.perf_counter() - t0, "tol": 1e-6,
                                  "within_tol": bool(ec["err"] <= 1e-6)}
        log("oracle check, colour transfer: FP64 marginal err on the exact cost %.3e" % ec["err"])
    if diff_x is not None:
        d = diff_x
        rows = []
        for k in (0, 37):
            Xk, Yk = d["X"][k].cpu().numpy(), d["Y"][k].cpu().numpy()
            fk, gk = d["f"][k].cpu().numpy(), d["g"][k].cpu().numpy()
            ox, oy = O.grad_points(0, Xk, Yk, d["scale"], d["eps"], fk, gk)
            gx, gy = d["dX"][k].cpu().numpy().astype(np.float64), d["dY"][k].cpu().numpy().astype(np.float64)
            ek = O.evaluate_points(0, Xk, Yk, d["scale"], d["eps"], O.normalize(d["a"][k].cpu().numpy()),
                                   O.normalize(d["b"][k].cpu().numpy()), fk, gk)
            rows.append({"problem": k,
                         "grad_X_rel_l2": float(np.linalg.norm(gx - ox) / np.linalg.norm(ox)),
                         "grad_Y_rel_l2": float(np.linalg.norm(gy - oy) / np.linalg.norm(oy)),
                         "fp64_marginal_err_exact_cost": ek["err"]})
            log("oracle check, diff loss problem %d: grad rel err %.2e / %.2e, FP64 marginal err %.3e"
                % (k, rows[-1]["grad_X_rel_l2"], rows[-1]["grad_Y_rel_l2"], ek["err"]))
        err["differentiable_loss"] = {"note": "backward at the GPU potentials against the oracle's envelope "
                                              "gradient on the exact FP64 cost; the forward solved the BF16x3 "
                                              "split cost, so its FP64 error on the exact cost is stated",
                                      "problems": rows}
    return cpu, err


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.with_copy:
        copy_calibration()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU row sharding is a design, "
              "not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_30267_amd import accsk
    from paper_2605_30267_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    accsk.lib()
    dev = torch.device("cuda:0")
    n = m = args.n
    log("generating gmm_dense n=m=%d" % n)
    p = W.gmm_dense(seed=2, n=n, m=m, eps=args.eps)
    C = torch.as_tensor(p["C32"], device=dev)
    a = torch.as_tensor(p["a"], dtype=torch.float64, device=dev)
    b = torch.as_tensor(p["b"], dtype=torch.float64, device=dev)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty(m, dtype=torch.float64, device=dev)

    def solve(eps, method):
        return accsk.solve_dense(C, a, b, eps, tol=1e-6, method=method, max_iter=1000000, f_out=f, g_out=g,
                                 flags=args.flags)[2]

    for _ in range(args.warmup):
        r = solve(args.eps, accsk.ACC)
        log("warmup: It %d err %.3e kernel %.2f ms" % (r["iters"], r["marginal_err"], r["kernel_ms"]))
    torch.cuda.synchronize()
    rs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rs.append(solve(args.eps, accsk.ACC))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    ok = all(r["converged"] == 1 for r in rs)
    solves_per_s = args.steps / dt
    steps_tot = sum(r["sinkhorn_steps"] for r in rs)
    kms_tot = sum(r["kernel_ms"] for r in rs)
    # Algorithmic bytes per Sinkhorn step: one read of C (n m 4 B).  Both
    # log-sum-exps of a step come from that one read (the column sums reuse the
    # row exponentials), so it is the method's minimum traffic.  The two-pass
    # figure (a row pass and a column pass, each streaming C) is reported beside
    # it for comparison with solvers that read C twice.
    alg_per_step = n * m * 4
    two_pass_per_step = 2 * n * m * 4
    alg_bytes = steps_tot * alg_per_step
    achieved = alg_bytes / (kms_tot * 1e-3) / 1e9
    two_pass_rate = steps_tot * two_pass_per_step / (kms_tot * 1e-3) / 1e9
    traffic, tinfo = traffic_from_profile()
    log("timed: %d solves in %.3f s, It %d, kernel avg %.3f ms, C read at %.1f GB/s (%.3f of 8 TB/s)"
        % (args.steps, dt, rs[0]["iters"], kms_tot / args.steps, achieved, achieved / HBM_PEAK_GBPS))

    # Measured read-stream bandwidth, outside the timed region: the references
    # the read rate of C is compared with beside the published peak.  Over
    # 1 GiB (four times the last-level cache) it is HBM's; re-reading C itself
    # (the solve's footprint, about the cache's size) it includes what the
    # cache keeps between passes.
    sbuf = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    stream_gbps = accsk.read_bandwidth(sbuf, reps=10)
    del sbuf
    stream_c_gbps = accsk.read_bandwidth(C, reps=20)
    log("read stream: %.1f GB/s over 1 GiB, %.1f GB/s re-reading C; C read by the solve at %.3f / %.3f of them"
        % (stream_gbps, stream_c_gbps, achieved / stream_gbps, achieved / stream_c_gbps))

    context = {}
    if args.context:
        for eps in (1e-2, 1e-3, 1e-4):
            row = {}
            for name, meth in (("acc", accsk.ACC), ("sinkhorn", accsk.SINKHORN)):
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                r = solve(eps, meth)
                torch.cuda.synchronize()
                s1 = time.perf_counter()
                row[name] = dict(iters=r["iters"], sinkhorn_steps=r["sinkhorn_steps"],
                                 fallback_steps=r["fallback_steps"], seconds=round(s1 - s0, 5),
                                 kernel_ms=round(r["kernel_ms"], 3), converged=r["converged"],
                                 us_per_step=round(1e3 * r["kernel_ms"] / r["sinkhorn_steps"], 2))
                log("context eps %g %s: It %d, %.4f s" % (eps, name, r["iters"], s1 - s0))
            row["speedup_acc_over_sinkhorn"] = round(row["sinkhorn"]["seconds"] / row["acc"]["seconds"], 2)
            context["eps=%g" % eps] = row

    color, color_x = color_bench(args, dev) if args.color else (None, None)
    diff, diff_x = diff_bench(args, dev) if args.diff else (None, None)
    small = small_batch_bench(args, dev) if args.small_batch else None
    fly = fly_mfma_bench(args, dev) if args.fly_mfma else None
    serving = serving_bench(args, dev) if args.serving else None
    paper = paper_bench(args, dev) if args.paper else None

    cpu = None
    oracle_error = None
    if args.cpu_baseline:
        r_head = solve(args.eps, accsk.ACC)
        fh, gh = f.cpu().numpy(), g.cpu().numpy()
        cpu, oracle_error = cpu_baseline_leg(args, p, steps_tot / args.steps, fh, gh, r_head, color_x, diff_x)

    out = {
        "metric": "solves/s to L1 marginal err<=1e-6 & % HBM roofline; p50/p99 batched latency",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "gmm_dense explicit FP32 cost n=m=%d, Acc-Sinkhorn, eps=%g, tol=1e-6"
                               % (n, args.eps), "n": n, "m": m, "eps": args.eps, "tol": 1e-6,
                   "method": "acc", "all_converged": ok, "iters": rs[0]["iters"],
                   "sinkhorn_steps": rs[0]["sinkhorn_steps"], "fallback_steps": rs[0]["fallback_steps"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": kernel_name(n),
                     "algorithmic_bytes_per_launch": alg_bytes / args.steps,
                     "algorithmic_bytes_per_step": alg_per_step, "reads_of_C_per_step": 1,
                     "steps_per_launch": steps_tot / args.steps,
                     "avg_launch_ms": kms_tot / args.steps,
                     "measured_read_stream_GBps": stream_gbps,
                     "frac_of_measured_stream": achieved / stream_gbps,
                     "measured_reread_of_C_GBps": stream_c_gbps,
                     "frac_of_measured_reread": achieved / stream_c_gbps,
                     "two_pass_bytes_per_step": two_pass_per_step,
                     "two_pass_rate_GBps": two_pass_rate},
        "cpu_baseline": cpu,
        "oracle_error": oracle_error,
        "context": context,
        "colour_transfer": color,
        "differentiable_loss": diff,
        "small_batch": small,
        "on_the_fly_mfma": fly,
        "serving": serving,
        "paper_experiments": paper,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
