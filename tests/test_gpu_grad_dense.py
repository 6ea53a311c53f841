"""Differentiation of the EOT value for explicit costs (eq:P-from-dual, envelope
theorem): accsk_backward_dense and the torch.autograd Function built on it.

At given potentials the gradient is a plain definition: dC = P with
P_ij = exp((f_i + g_j - C_ij)/eps), and the marginal gradients are
(f - <f, a/sum a>)/sum a (and likewise for b).  The kernel forms the argument
and the exponential in FP64 and rounds P once to FP32, so dC agrees with the
oracle's FP64 plan to one FP32 rounding (2^-24 relative); the marginal
gradients are FP64 throughout.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_30267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("n,m,eps", [(300, 2500, 3e-2), (5000, 37, 5e-2), (1, 1, 1e-1)])
def test_backward_dense_against_oracle(torch_gpu, n, m, eps):
    """Potentials from the oracle; rows beyond the 4096-row grid (n = 5000), a ragged last column block."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    p = W.random_dense(seed=n + m, n=n, m=m, eps=eps)
    rng = np.random.default_rng(n)
    a_raw, b_raw = p["a"] * rng.uniform(0.5, 2.0), p["b"] * 3.0
    C64 = p["C32"].astype(np.float64)
    o = O.solve(C64, a_raw, b_raw, eps, tol=1e-11, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    fo, go = o["f"], o["g"]
    gsc = 1.75
    print("case backward dense", n, m, eps, flush=True)
    dC, da, db = accsk.backward_dense(_dev(torch, p["C32"], torch.float32), _dev(torch, a_raw, torch.float64),
                                      _dev(torch, b_raw, torch.float64), _dev(torch, fo, torch.float64),
                                      _dev(torch, go, torch.float64), eps,
                                      grad_scale=torch.tensor(gsc, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    P = O.plan(C64, eps, fo, go)
    got = dC.cpu().numpy().astype(np.float64) / gsc
    assert np.all(np.abs(got - P) <= 2.0 ** -23 * np.abs(P) + 1e-300)
    ra, rb = O.grad_marginals(fo, go, a_raw, b_raw)
    assert np.allclose(da.cpu().numpy() / gsc, ra, rtol=1e-12, atol=1e-14 * np.abs(fo).max() / a_raw.sum())
    assert np.allclose(db.cpu().numpy() / gsc, rb, rtol=1e-12, atol=1e-14 * np.abs(go).max() / b_raw.sum())
    # marginals only: dC not written
    _, da2, db2 = accsk.backward_dense(_dev(torch, p["C32"], torch.float32), _dev(torch, a_raw, torch.float64),
                                       _dev(torch, b_raw, torch.float64), _dev(torch, fo, torch.float64),
                                       _dev(torch, go, torch.float64), eps, cost=False)
    assert np.allclose(da2.cpu().numpy(), ra, rtol=1e-12, atol=1e-14 * np.abs(fo).max() / a_raw.sum())


def test_eot_loss_dense_autograd(torch_gpu):
    """torch.autograd through the library on an explicit cost: value and gradients against the
    oracle's solve (the forward converges to tol 1e-9, the oracle to 1e-11)."""
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    n, m, eps = 120, 90, 5e-2
    p = W.random_dense(seed=5, n=n, m=m, eps=eps)
    rng = np.random.default_rng(6)
    a_raw, b_raw = rng.uniform(0.5, 1.5, n), rng.uniform(0.5, 1.5, m)
    C = _dev(torch, p["C32"], torch.float32).requires_grad_(True)
    a = _dev(torch, a_raw, torch.float64).requires_grad_(True)
    b = _dev(torch, b_raw, torch.float64).requires_grad_(True)
    print("case eot_loss_dense", n, m, eps, flush=True)
    val = accsk.eot_loss_dense(C, a, b, eps, tol=1e-9)
    (2.5 * val).backward()
    torch.cuda.synchronize()
    C64 = p["C32"].astype(np.float64)
    o = O.solve(C64, a_raw, b_raw, eps, tol=1e-11, method=O.ACC, mu0=0.25, m0=5, w_rule=O.W_Y_CONTINUOUS)
    ev = O.evaluate(C64, eps, a_raw / a_raw.sum(), b_raw / b_raw.sum(), o["f"], o["g"])
    assert abs(val.item() - ev["dual"]) <= 1e-6 * eps
    P = O.plan(C64, eps, o["f"], o["g"])
    ra, rb = O.grad_marginals(o["f"], o["g"], a_raw, b_raw)
    for got, ref in ((C.grad, P), (a.grad, ra), (b.grad, rb)):
        got = got.detach().cpu().numpy().astype(np.float64) / 2.5
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
