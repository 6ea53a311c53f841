"""Host-side checks of the C-ABI (no GPU needed).

* libaccsk.so loads and exports every entry point declared in include/accsk.h.
* Argument validation happens on the host before any device work: invalid
  scalars and shapes return the documented status with null device pointers.
* The ctypes structures match the header's field lists.
"""
import ctypes
import os
import re

import pytest

from paper_2605_30267_amd import accsk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(accsk.LIB_PATH):
        pytest.skip("libaccsk.so not built")
    return accsk.lib()


def test_exports_every_declared_symbol(lib):
    names = accsk.symbols_declared()
    assert "accsk_solve_dense" in names and "accsk_solve_batch" in names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_fields_match_header():
    text = open(os.path.join(ROOT, "include", "accsk.h")).read()

    def fields(struct_name):
        body = re.search(r"typedef struct (?:\w+ )?\{([^{}]*)\} %s;" % struct_name, text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                out.append(part.strip().split()[-1].lstrip("*"))
        return out

    assert fields("accsk_params") == [f for f, _ in accsk.Params._fields_]
    assert fields("accsk_result") == [f for f, _ in accsk.Result._fields_]
    assert fields("accsk_problem") == [f for f, _ in accsk.Problem._fields_]
    assert fields("accsk_request") == [f for f, _ in accsk.Request._fields_]


def test_defaults(lib):
    p = accsk.default_params()
    assert p.method == accsk.ACC and p.w_rule == accsk.W_Y_CONTINUOUS
    assert 0 < p.mu0 < 1 and p.m0 >= 1 and p.tol == 1e-6
    assert lib.accsk_status_string(accsk.SHAPE).decode().startswith("unsupported")


def _solve_dense_raw(lib, n, m, ldc, eps=1e-2, tol=1e-6, method=1, mu0=0.25, m0=5, ptr=1):
    p = accsk.default_params(eps=eps, tol=tol, method=method, mu0=mu0, m0=m0)
    r = accsk.Result()
    fake = ctypes.c_void_p(ptr)
    return lib.accsk_solve_dense(fake, n, m, ldc, fake, fake, ctypes.byref(p), fake, fake, ctypes.byref(r), None)


def test_host_validation_dense(lib):
    assert _solve_dense_raw(lib, 4, 4, 4, eps=-1.0) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 4, 4, 4, eps=float("nan")) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 4, 4, 4, tol=0.0) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 4, 4, 4, mu0=1.0) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 4, 4, 4, m0=0) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 4, 4, 4, method=7) == accsk.INVALID_ARG
    assert _solve_dense_raw(lib, 0, 4, 4) == accsk.SHAPE
    assert _solve_dense_raw(lib, 4, 4, 3) == accsk.SHAPE
    assert _solve_dense_raw(lib, 4, 4, 4, ptr=0) == accsk.INVALID_ARG


def test_host_validation_batch(lib):
    p = accsk.default_params()
    res = (accsk.Result * 1)()
    arr = (accsk.Problem * 1)()
    arr[0] = accsk.Problem(1, 4, 4, 4, 1, 1, 1, 1, 1e-2)
    bad = accsk.Problem(1, 4, 9000, 9000, 1, 1, 1, 1, 1e-2)
    arr2 = (accsk.Problem * 1)(bad)
    assert lib.accsk_solve_batch(arr2, 1, ctypes.byref(p), res, None) == accsk.SHAPE
    arr3 = (accsk.Problem * 1)(accsk.Problem(1, 4, 4, 4, 1, 1, 1, 1, 0.0))
    assert lib.accsk_solve_batch(arr3, 1, ctypes.byref(p), res, None) == accsk.INVALID_ARG
    assert lib.accsk_solve_batch(arr, 0, ctypes.byref(p), res, None) == accsk.OK


def test_host_validation_batch_strided(lib):
    p = accsk.default_params()
    res = (accsk.Result * 2)()
    fake = 4096  # never dereferenced: every case fails validation on the host
    f = lib.accsk_solve_batch_strided
    assert f(None, 2, 4, 4, 4, 16, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.INVALID_ARG
    assert f(fake, -1, 4, 4, 4, 16, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.INVALID_ARG
    assert f(fake, 0, 4, 4, 4, 16, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.OK
    assert f(fake, 2, 4, 4, 3, 16, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.SHAPE
    assert f(fake, 2, 4, 4, 4, 15, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.SHAPE
    assert f(fake, 2, 0, 4, 4, 16, fake, fake, None, ctypes.byref(p), fake, fake, res, None) == accsk.SHAPE
    bad_eps = (ctypes.c_double * 2)(1e-2, -1.0)
    assert f(fake, 2, 4, 4, 4, 16, fake, fake, bad_eps, ctypes.byref(p), fake, fake, res, None) == accsk.INVALID_ARG


def test_host_validation_server(lib):
    accsk._register_server(lib)
    h = ctypes.c_void_p()
    for kw, budget in ((dict(tol=0.0), 1 << 20), (dict(split=1), 1 << 20), (dict(method=5), 1 << 20), ({}, 0)):
        p = accsk.default_params(**kw)
        assert lib.accsk_server_create(budget, 0, ctypes.byref(p), ctypes.byref(h)) == accsk.INVALID_ARG
        assert not h.value
    req = accsk.Request()
    t = ctypes.c_uint64()
    assert lib.accsk_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == accsk.INVALID_ARG
    done = ctypes.c_int()
    assert lib.accsk_server_poll(None, 1, None, ctypes.byref(done), None) == accsk.INVALID_ARG
    assert lib.accsk_server_destroy(None) == accsk.INVALID_ARG
    t0 = lib.accsk_clock_seconds()
    assert lib.accsk_clock_seconds() >= t0 > 0


def test_results_as_arrays_layout():
    """The numpy view of a Result array reads every field at the ctypes offsets."""
    r = (accsk.Result * 3)()
    r[1].iters, r[1].eot_value, r[2].status, r[2].converged, r[0].kernel_ms = 7, 1.5, 4, 1, 2.5
    r[0].restarts, r[2].dual_fval = 3, -0.25
    d = accsk.results_as_arrays(r)
    for k in range(3):
        for name, _ in accsk.Result._fields_:
            assert d[name][k] == getattr(r[k], name), (k, name)


def test_host_validation_trace(lib):
    """The per-step error trace: one problem per call, a buffer for a positive length, not on a server."""
    fake = 4096  # never dereferenced: every case fails validation on the host
    r = accsk.Result()
    p = accsk.default_params(trace_len=-1)
    assert lib.accsk_solve_dense(fake, 4, 4, 4, fake, fake, ctypes.byref(p), fake, fake, ctypes.byref(r),
                                 None) == accsk.INVALID_ARG
    p = accsk.default_params(trace_len=5)  # no buffer
    assert lib.accsk_solve_dense(fake, 4, 4, 4, fake, fake, ctypes.byref(p), fake, fake, ctypes.byref(r),
                                 None) == accsk.INVALID_ARG
    p = accsk.default_params(err_trace=fake, trace_len=5)
    res = (accsk.Result * 2)()
    arr = (accsk.Problem * 2)(accsk.Problem(fake, 4, 4, 4, fake, fake, fake, fake, 1e-2),
                              accsk.Problem(fake, 4, 4, 4, fake, fake, fake, fake, 1e-2))
    assert lib.accsk_solve_batch(arr, 2, ctypes.byref(p), res, None) == accsk.INVALID_ARG
    pl = accsk._points_lib()
    assert pl.accsk_solve_points_batched(fake, fake, 2, 4, 4, 3, 0, 1.0, fake, fake, ctypes.byref(p), fake, fake,
                                         res, None) == accsk.INVALID_ARG
    accsk._register_server(lib)
    h = ctypes.c_void_p()
    assert lib.accsk_server_create(1 << 20, 0, ctypes.byref(p), ctypes.byref(h)) == accsk.INVALID_ARG


def test_host_validation_workspace_bytes(lib):
    out = ctypes.c_size_t(0)
    assert lib.accsk_workspace_bytes(4, 4, 1, None) == accsk.INVALID_ARG
    assert lib.accsk_workspace_bytes(4, 4, 0, ctypes.byref(out)) == accsk.INVALID_ARG
    assert lib.accsk_workspace_bytes(0, 4, 1, ctypes.byref(out)) == accsk.SHAPE
    assert lib.accsk_workspace_bytes(4, 0, 1, ctypes.byref(out)) == accsk.SHAPE


def test_host_validation_read_bandwidth(lib):
    out = ctypes.c_double(0.0)
    f = lib.accsk_read_bandwidth
    assert f(None, 1 << 20, 1, ctypes.byref(out), None) == accsk.INVALID_ARG
    assert f(4096, 1 << 20, 0, ctypes.byref(out), None) == accsk.INVALID_ARG
    assert f(4096, 8, 1, ctypes.byref(out), None) == accsk.INVALID_ARG
    assert f(4097, 1 << 20, 1, ctypes.byref(out), None) == accsk.INVALID_ARG
    assert f(4096, 1 << 20, 1, None, None) == accsk.INVALID_ARG


def test_host_validation_exp_rate(lib):
    out = ctypes.c_double(0.0)
    assert lib.accsk_exp_rate(0, ctypes.byref(out), None) == accsk.INVALID_ARG
    assert lib.accsk_exp_rate(1, None, None) == accsk.INVALID_ARG


def test_host_validation_noalloc(lib):
    """The allocation-free dense solve validates on the host before touching the device."""
    f = lib.accsk_solve_dense_noalloc
    r = accsk.Result()
    fake = ctypes.c_void_p(4096)  # never dereferenced

    def call(n, m, ldc, ptr=fake, **kw):
        p = accsk.default_params(**kw)
        return f(ptr, n, m, ldc, fake, fake, ctypes.byref(p), fake, fake, ctypes.byref(r), None)

    assert call(4, 4, 4, ptr=None) == accsk.INVALID_ARG
    assert call(4, 4, 4, eps=-1.0) == accsk.INVALID_ARG
    assert call(4, 4, 4, tol=0.0) == accsk.INVALID_ARG
    assert call(0, 4, 4) == accsk.SHAPE
    assert call(4, 4, 3) == accsk.SHAPE
    assert call(4, 9000, 9000) == accsk.SHAPE
    assert r.status == accsk.INVALID_ARG and r.converged == 0


def test_host_validation_async(lib):
    """Stream-ordered entry points: a missing record array or bad shapes fail on the host."""
    fake = ctypes.c_void_p(4096)  # never dereferenced
    p = accsk.default_params()
    f = lib.accsk_solve_dense_async
    assert f(fake, 4, 4, 4, fake, fake, ctypes.byref(p), fake, fake, None, None) == accsk.INVALID_ARG
    assert f(fake, 0, 4, 4, fake, fake, ctypes.byref(p), fake, fake, fake, None) == accsk.SHAPE
    assert f(fake, 4, 4, 3, fake, fake, ctypes.byref(p), fake, fake, fake, None) == accsk.SHAPE
    bad = accsk.default_params(eps=-1.0)
    assert f(fake, 4, 4, 4, fake, fake, ctypes.byref(bad), fake, fake, fake, None) == accsk.INVALID_ARG
    g = lib.accsk_solve_batch_strided_async
    assert g(fake, 2, 4, 4, 4, 16, fake, fake, None, ctypes.byref(p), fake, fake, None, None) == accsk.INVALID_ARG
    assert g(fake, 2, 4, 4, 3, 16, fake, fake, None, ctypes.byref(p), fake, fake, fake, None) == accsk.SHAPE
    h = accsk._points_lib().accsk_solve_points_batched_async
    assert h(fake, fake, 2, 4, 4, 3, 0, 1.0, fake, fake, ctypes.byref(p), fake, fake, None, None) == accsk.INVALID_ARG
    assert h(fake, fake, 2, 4, 4, 0, 0, 1.0, fake, fake, ctypes.byref(p), fake, fake, fake, None) == accsk.SHAPE


def test_host_validation_backward_dense(lib):
    """accsk_backward_dense: missing arrays, eps and shapes fail before any device work."""
    fake = ctypes.c_void_p(4096)  # never dereferenced
    f = accsk._points_lib().accsk_backward_dense
    # (C, n, m, ldc, eps, a, b, f, g, grad_scale, dC, lddc, da, db, stream)
    assert f(fake, 4, 5, 5, 0.1, fake, fake, None, fake, None, fake, 5, None, None, None) == accsk.INVALID_ARG
    assert f(None, 4, 5, 5, 0.1, fake, fake, fake, fake, None, fake, 5, None, None, None) == accsk.INVALID_ARG
    assert f(fake, 4, 5, 5, 0.1, None, fake, fake, fake, None, None, 5, fake, None, None) == accsk.INVALID_ARG
    assert f(fake, 4, 5, 5, 0.0, fake, fake, fake, fake, None, fake, 5, None, None, None) == accsk.INVALID_ARG
    assert f(fake, 4, 5, 4, 0.1, fake, fake, fake, fake, None, fake, 5, None, None, None) == accsk.SHAPE
    assert f(fake, 4, 5, 5, 0.1, fake, fake, fake, fake, None, fake, 4, None, None, None) == accsk.SHAPE
    assert f(fake, 0, 5, 5, 0.1, fake, fake, fake, fake, None, fake, 5, None, None, None) == accsk.SHAPE


def test_host_validation_cost_points_batched(lib):
    fake = ctypes.c_void_p(4096)  # never dereferenced
    f = accsk._points_lib().accsk_cost_points_batched
    # (X, Y, batch, n, m, d, kind, cost_scale, split, C, ldc, stream)
    assert f(fake, fake, 0, 4, 5, 3, 0, 1.0, 3, fake, 5, None) == accsk.INVALID_ARG
    assert f(fake, fake, 2, 4, 5, 3, 0, 1.0, 3, None, 5, None) == accsk.INVALID_ARG
    assert f(fake, fake, 2, 4, 5, 3, 0, 1.0, 3, fake, 4, None) == accsk.SHAPE
    assert f(fake, fake, 2, 4, 5, 513, 0, 1.0, 3, fake, 5, None) == accsk.SHAPE
    assert f(fake, fake, 2, 4, 5, 3, 0, 1.0, 1, fake, 5, None) == accsk.INVALID_ARG
