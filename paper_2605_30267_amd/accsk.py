"""ctypes binding of libaccsk (the HIP/gfx950 Acc-Sinkhorn library).

Argument marshalling only: every step of every solve runs in the library's
kernels.  Tensors must already live on the current HIP device; work is enqueued
on torch's current stream.  The library is loaded on first use and its absence
is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaccsk.so")

OK, INVALID_ARG, SHAPE, NONFINITE, NOT_CONVERGED, DIVERGED, OOM, HIP_ERROR, BUSY = range(9)
SINKHORN, ACC = 0, 1
W_LITERAL, W_Y_CONTINUOUS = 0, 1
SQEUCLID, COSINE = 0, 1
FLAG_NO_COST = 1
FLAG_NO_SERPENTINE = 2
FLAG_ON_THE_FLY = 4
FLAG_RESTART = 8
FLAG_CONDITIONS = 16


class AccskError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, status_string(status), status))


class Params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("w_rule", ctypes.c_int32), ("eps", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int64), ("mu0", ctypes.c_double),
                ("m0", ctypes.c_int64), ("split", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("err_trace", ctypes.c_void_p), ("trace_len", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("sinkhorn_steps", ctypes.c_int64),
                ("fallback_steps", ctypes.c_int64), ("fval_increases", ctypes.c_int64),
                ("restarts", ctypes.c_int64), ("cond1_violations", ctypes.c_int64),
                ("cond2_violations", ctypes.c_int64), ("lyap_increases", ctypes.c_int64),
                ("marginal_err", ctypes.c_double),
                ("eot_value", ctypes.c_double), ("transport_cost", ctypes.c_double),
                ("dual_fval", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Problem(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("f", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("eps", ctypes.c_double)]


_lib = None
_lock = threading.Lock()
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def lib():
    """Load libaccsk.so (built in-tree by ``paper_2605_30267_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libaccsk.so is not built (%s); run python -m paper_2605_30267_amd.build"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.accsk_default_params.argtypes = [ctypes.POINTER(Params)]
        L.accsk_default_params.restype = None
        L.accsk_status_string.argtypes = [ctypes.c_int]
        L.accsk_status_string.restype = ctypes.c_char_p
        L.accsk_version.argtypes = []
        L.accsk_version.restype = ctypes.c_char_p
        L.accsk_solve_dense.argtypes = [_vp, _i64, _i64, _i64, _vp, _vp, ctypes.POINTER(Params), _vp, _vp,
                                        ctypes.POINTER(Result), _vp]
        L.accsk_solve_dense.restype = ctypes.c_int
        L.accsk_solve_dense_noalloc.argtypes = L.accsk_solve_dense.argtypes
        L.accsk_solve_dense_noalloc.restype = ctypes.c_int
        L.accsk_solve_dense_async.argtypes = [_vp, _i64, _i64, _i64, _vp, _vp, ctypes.POINTER(Params), _vp, _vp,
                                              _vp, _vp]
        L.accsk_solve_dense_async.restype = ctypes.c_int
        L.accsk_plan_dense.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _i64, _i64, _vp, _i64, _vp]
        L.accsk_plan_dense.restype = ctypes.c_int
        L.accsk_eval_dense.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _vp, _vp,
                                       ctypes.POINTER(ctypes.c_double), _vp]
        L.accsk_eval_dense.restype = ctypes.c_int
        L.accsk_solve_batch.argtypes = [ctypes.POINTER(Problem), _i64, ctypes.POINTER(Params),
                                        ctypes.POINTER(Result), _vp]
        L.accsk_solve_batch.restype = ctypes.c_int
        L.accsk_solve_batch_strided.argtypes = [_vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _vp,
                                                ctypes.POINTER(Params), _vp, _vp, ctypes.POINTER(Result), _vp]
        L.accsk_solve_batch_strided.restype = ctypes.c_int
        L.accsk_solve_batch_strided_async.argtypes = [_vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _vp,
                                                      ctypes.POINTER(Params), _vp, _vp, _vp, _vp]
        L.accsk_solve_batch_strided_async.restype = ctypes.c_int
        L.accsk_workspace_bytes.argtypes = [_i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)]
        L.accsk_workspace_bytes.restype = ctypes.c_int
        L.accsk_read_bandwidth.argtypes = [_vp, _i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _vp]
        L.accsk_read_bandwidth.restype = ctypes.c_int
        L.accsk_exp_rate.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _vp]
        L.accsk_exp_rate.restype = ctypes.c_int
        _lib = L
        return L


def status_string(status):
    try:
        return lib().accsk_status_string(int(status)).decode()
    except Exception:  # library missing: still produce a message
        return "status %d" % status


def default_params(**kw):
    p = Params()
    lib().accsk_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(p, k):
            raise TypeError("unknown parameter %r" % k)
        setattr(p, k, v)
    return p


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(t, dtype, name, ndim=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dims" % (name, ndim))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _trace_buffer(p, trace, max_iter, device):
    """Device FP64 buffer for the per-step error trace (one entry per Sinkhorn step), or None."""
    if not trace:
        return None
    import torch
    buf = torch.full((int(max_iter) + 1,), float("nan"), dtype=torch.float64, device=device)
    p.err_trace = buf.data_ptr()
    p.trace_len = buf.numel()
    return buf


def solve_dense(C, a, b, eps, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None,
                w_rule=None, flags=0, f_out=None, g_out=None, raise_on_error=True, trace=False):
    """Solve EOT on a dense FP32 cost (device).  Returns (f, g, result dict).

    C: float32 [n, m] (row stride used as leading dimension, unit column stride);
    a: float64 [n], b: float64 [m] (positive; normalized inside).
    trace=True adds result["trace"]: the L1 marginal error of every Sinkhorn step (numpy).
    """
    return _solve_dense_call("accsk_solve_dense", C, a, b, eps, tol, method, max_iter, mu0, m0, w_rule, flags,
                             f_out, g_out, raise_on_error, trace)


def solve_dense_noalloc(C, a, b, eps, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None,
                        w_rule=None, flags=0, f_out=None, g_out=None, raise_on_error=True, trace=False):
    """solve_dense through accsk_solve_dense_noalloc: the library allocates no device memory (its
    workspace is a fixed per-device array).  Pass f_out / g_out to avoid torch allocations too."""
    return _solve_dense_call("accsk_solve_dense_noalloc", C, a, b, eps, tol, method, max_iter, mu0, m0, w_rule,
                             flags, f_out, g_out, raise_on_error, trace)


def _solve_dense_call(entry, C, a, b, eps, tol, method, max_iter, mu0, m0, w_rule, flags, f_out, g_out,
                      raise_on_error, trace):
    import torch
    _check_dev(C, torch.float32, "C", 2)
    _check_dev(a, torch.float64, "a", 1)
    _check_dev(b, torch.float64, "b", 1)
    if C.stride(1) != 1:
        raise ValueError("C must have unit column stride")
    n, m = C.shape
    a = a.contiguous()
    b = b.contiguous()
    if f_out is None:
        f_out = torch.empty(n, dtype=torch.float64, device=C.device)
    if g_out is None:
        g_out = torch.empty(m, dtype=torch.float64, device=C.device)
    p = default_params(method=method, eps=float(eps), tol=float(tol), max_iter=int(max_iter), mu0=mu0,
                       m0=m0, w_rule=w_rule, flags=int(flags))
    tbuf = _trace_buffer(p, trace, max_iter, C.device)
    r = Result()
    st = getattr(lib(), entry)(_ptr(C), n, m, C.stride(0), _ptr(a), _ptr(b), ctypes.byref(p), _ptr(f_out),
                               _ptr(g_out), ctypes.byref(r), _stream_ptr())
    if raise_on_error and st not in (OK, NOT_CONVERGED):
        raise AccskError(st, entry)
    d = r.to_dict()
    d["status"] = st
    if tbuf is not None:
        d["trace"] = tbuf[:max(0, min(r.sinkhorn_steps, tbuf.numel()))].cpu().numpy()
    return f_out, g_out, d


def solve_batch(problems, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None, w_rule=None, flags=0,
                raise_on_error=True):
    """Solve independent dense problems, one workgroup each.

    problems: list of (C float32 [n,m] device, a float64 [n], b float64 [m], eps).
    Returns (list of (f, g), list of result dicts, batch status).
    """
    import torch
    k = len(problems)
    arr = (Problem * k)()
    outs = []
    keep = []
    for idx, (C, a, b, eps) in enumerate(problems):
        _check_dev(C, torch.float32, "C", 2)
        _check_dev(a, torch.float64, "a", 1)
        _check_dev(b, torch.float64, "b", 1)
        if C.stride(1) != 1:
            raise ValueError("C must have unit column stride")
        n, m = C.shape
        a = a.contiguous()
        b = b.contiguous()
        f = torch.empty(n, dtype=torch.float64, device=C.device)
        g = torch.empty(m, dtype=torch.float64, device=C.device)
        keep += [a, b]
        outs.append((f, g))
        arr[idx] = Problem(C.data_ptr(), n, m, C.stride(0), a.data_ptr(), b.data_ptr(), f.data_ptr(),
                           g.data_ptr(), float(eps))
    p = default_params(method=method, tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0, w_rule=w_rule,
                       flags=int(flags))
    res = (Result * k)()
    st = lib().accsk_solve_batch(arr, k, ctypes.byref(p), res, _stream_ptr())
    if raise_on_error and st not in (OK, NOT_CONVERGED):
        raise AccskError(st, "accsk_solve_batch")
    return outs, [r.to_dict() for r in res], st


def workspace_bytes(n, m, count=1):
    """Upper bound of the device workspace of a dense or batched solve (bytes)."""
    out = ctypes.c_size_t(0)
    st = lib().accsk_workspace_bytes(int(n), int(m), int(count), ctypes.byref(out))
    if st != OK:
        raise AccskError(st, "accsk_workspace_bytes")
    return out.value


def read_bandwidth(buf, reps=10):
    """Measured HBM read bandwidth (GB/s) of a read-only stream over the device tensor buf."""
    out = ctypes.c_double(0.0)
    st = lib().accsk_read_bandwidth(_ptr(buf), buf.numel() * buf.element_size(), int(reps), ctypes.byref(out),
                                    _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_read_bandwidth")
    return out.value


def exp_rate(reps=5):
    """Measured FP32 exponential (v_exp_f32) throughput of the device, in exponentials per second."""
    out = ctypes.c_double(0.0)
    st = lib().accsk_exp_rate(int(reps), ctypes.byref(out), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_exp_rate")
    return out.value


def solve_batch_strided(C, a, b, eps, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None, w_rule=None,
                        flags=0, raise_on_error=True):
    """Solve B problems of one shape held in strided tensors (one call, no per-problem work in Python).

    C: float32 [B, n, m] on the device, unit column stride; a: float64 [B, n]; b: float64 [B, m];
    eps: a float or a sequence of B floats.  Returns (f [B, n], g [B, m], results, status) with
    results a dict of numpy arrays of length B, one per result field.
    """
    import torch
    _check_dev(C, torch.float32, "C", 3)
    _check_dev(a, torch.float64, "a", 2)
    _check_dev(b, torch.float64, "b", 2)
    if C.stride(2) != 1:
        raise ValueError("C must have unit column stride")
    B, n, m = C.shape
    if tuple(a.shape) != (B, n) or tuple(b.shape) != (B, m):
        raise ValueError("a must be [B, n] and b [B, m]")
    a = a.contiguous()
    b = b.contiguous()
    f = torch.empty((B, n), dtype=torch.float64, device=C.device)
    g = torch.empty((B, m), dtype=torch.float64, device=C.device)
    if isinstance(eps, (int, float)):
        p = default_params(eps=float(eps), method=method, tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0,
                           w_rule=w_rule, flags=int(flags))
        eps_arr = None
    else:
        p = default_params(method=method, tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0, w_rule=w_rule,
                           flags=int(flags))
        if len(eps) != B:
            raise ValueError("eps must have one value per problem")
        eps_arr = (ctypes.c_double * B)(*[float(e) for e in eps])
    res = (Result * B)()
    st = lib().accsk_solve_batch_strided(_ptr(C), B, n, m, C.stride(1), C.stride(0), _ptr(a), _ptr(b), eps_arr,
                                         ctypes.byref(p), _ptr(f), _ptr(g), res, _stream_ptr())
    if raise_on_error and st not in (OK, NOT_CONVERGED):
        raise AccskError(st, "accsk_solve_batch_strided")
    return f, g, results_as_arrays(res), st


def result_records(count, device):
    """Device memory for `count` accsk_result records (the stream-ordered entry points write them)."""
    import torch
    return torch.empty(count * ctypes.sizeof(Result), dtype=torch.uint8, device=device)


def read_records(rec):
    """Host copy of device result records as a list of dicts (the copy follows the stream's work)."""
    raw = rec.cpu().numpy().tobytes()
    sz = ctypes.sizeof(Result)
    return [Result.from_buffer_copy(raw, k * sz).to_dict() for k in range(len(raw) // sz)]


def solve_dense_async(C, a, b, eps, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None, w_rule=None,
                      flags=0, f_out=None, g_out=None, rec=None):
    """Stream-ordered solve_dense: enqueues the solve and returns (f, g, rec) at once; rec holds the
    device result record (read it with read_records after the stream has passed the work)."""
    import torch
    _check_dev(C, torch.float32, "C", 2)
    _check_dev(a, torch.float64, "a", 1)
    _check_dev(b, torch.float64, "b", 1)
    if C.stride(1) != 1:
        raise ValueError("C must have unit column stride")
    n, m = C.shape
    if not (a.is_contiguous() and b.is_contiguous()):
        raise ValueError("a and b must be contiguous (the call returns before the solve reads them)")
    if f_out is None:
        f_out = torch.empty(n, dtype=torch.float64, device=C.device)
    if g_out is None:
        g_out = torch.empty(m, dtype=torch.float64, device=C.device)
    if rec is None:
        rec = result_records(1, C.device)
    p = default_params(method=method, eps=float(eps), tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0,
                       w_rule=w_rule, flags=int(flags))
    st = lib().accsk_solve_dense_async(_ptr(C), n, m, C.stride(0), _ptr(a), _ptr(b), ctypes.byref(p),
                                       _ptr(f_out), _ptr(g_out), _ptr(rec), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_solve_dense_async")
    return f_out, g_out, rec


def solve_batch_strided_async(C, a, b, eps, tol=1e-6, method=ACC, max_iter=100000, mu0=None, m0=None,
                              w_rule=None, flags=0, rec=None):
    """Stream-ordered solve_batch_strided (eps: one float): returns (f [B, n], g [B, m], rec) at once."""
    import torch
    _check_dev(C, torch.float32, "C", 3)
    _check_dev(a, torch.float64, "a", 2)
    _check_dev(b, torch.float64, "b", 2)
    if C.stride(2) != 1 or not (a.is_contiguous() and b.is_contiguous()):
        raise ValueError("C must have unit column stride, a and b must be contiguous")
    B, n, m = C.shape
    f = torch.empty((B, n), dtype=torch.float64, device=C.device)
    g = torch.empty((B, m), dtype=torch.float64, device=C.device)
    if rec is None:
        rec = result_records(B, C.device)
    p = default_params(eps=float(eps), method=method, tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0,
                       w_rule=w_rule, flags=int(flags))
    st = lib().accsk_solve_batch_strided_async(_ptr(C), B, n, m, C.stride(1), C.stride(0), _ptr(a), _ptr(b), None,
                                               ctypes.byref(p), _ptr(f), _ptr(g), _ptr(rec), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_solve_batch_strided_async")
    return f, g, rec


def results_as_arrays(res):
    """A ctypes array of Result as a dict of numpy arrays, one per field (no per-problem objects)."""
    import numpy as np
    kinds = {ctypes.c_int64: "<i8", ctypes.c_double: "<f8", ctypes.c_int32: "<i4"}
    dt = np.dtype([(k, kinds[t]) for k, t in Result._fields_], align=True)
    assert dt.itemsize == ctypes.sizeof(Result)
    view = np.frombuffer(res, dtype=dt)
    return {k: view[k].copy() for k, _ in Result._fields_}


def plan_dense(C, f, g, eps, row0=0, rows=None, out=None):
    """FP32 rows of the plan P_ij = exp((f_i + g_j - C_ij)/eps)."""
    import torch
    n, m = C.shape
    rows = n - row0 if rows is None else rows
    if out is None:
        out = torch.empty((rows, m), dtype=torch.float32, device=C.device)
    st = lib().accsk_plan_dense(_ptr(C), n, m, C.stride(0), float(eps), _ptr(f), _ptr(g), int(row0), int(rows),
                                _ptr(out), out.stride(0), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_plan_dense")
    return out


def eval_dense(C, a, b, f, g, eps):
    """FP64-accumulated evaluation: dict(row_err, col_err, dual, cost, mass)."""
    n, m = C.shape
    out = (ctypes.c_double * 5)()
    st = lib().accsk_eval_dense(_ptr(C), n, m, C.stride(0), float(eps), _ptr(a), _ptr(b), _ptr(f), _ptr(g),
                                out, _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_eval_dense")
    return dict(row_err=out[0], col_err=out[1], dual=out[2], cost=out[3], mass=out[4])


def symbols_declared():
    """Names of the entry points declared in include/accsk.h (parsed from the header)."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "accsk.h")
    text = open(hdr).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)  # declarations only, not comments
    return sorted(set(re.findall(r"^[a-z_][a-z_0-9 \t*]*?\b(accsk_[a-z_0-9]+)\s*\(", text, re.M)))


def _register_points(L):
    if getattr(L, "_points_ready", False):
        return
    L.accsk_cost_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _dbl, ctypes.c_int, _vp, _i64, _vp]
    L.accsk_cost_points.restype = ctypes.c_int
    L.accsk_cost_points_batched.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.c_int, _dbl, ctypes.c_int, _vp,
                                            _i64, _vp]
    L.accsk_cost_points_batched.restype = ctypes.c_int
    L.accsk_solve_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _dbl, _vp, _vp,
                                     ctypes.POINTER(Params), _vp, _vp, ctypes.POINTER(Result), _vp]
    L.accsk_solve_points.restype = ctypes.c_int
    L.accsk_solve_points_batched.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.c_int, _dbl, _vp, _vp,
                                             ctypes.POINTER(Params), _vp, _vp, ctypes.POINTER(Result), _vp]
    L.accsk_solve_points_batched.restype = ctypes.c_int
    L.accsk_solve_points_batched_async.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.c_int, _dbl, _vp, _vp,
                                                   ctypes.POINTER(Params), _vp, _vp, _vp, _vp]
    L.accsk_solve_points_batched_async.restype = ctypes.c_int
    L.accsk_backward_points.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.c_int, _dbl, _dbl, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.accsk_backward_points.restype = ctypes.c_int
    L.accsk_backward_dense.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                       _vp]
    L.accsk_backward_dense.restype = ctypes.c_int
    L.accsk_cost_max_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, ctypes.POINTER(_dbl), _vp]
    L.accsk_cost_max_points.restype = ctypes.c_int
    L.accsk_plan_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _dbl, _dbl, _vp, _vp, _i64, _i64, _vp,
                                    _i64, _vp]
    L.accsk_plan_points.restype = ctypes.c_int
    L.accsk_barycentric_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _dbl, _dbl, _vp, _vp, _vp, _vp]
    L.accsk_barycentric_points.restype = ctypes.c_int
    L.accsk_topk_points.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _dbl, _dbl, _vp, _vp, ctypes.c_int,
                                    _vp, _vp, _vp]
    L.accsk_topk_points.restype = ctypes.c_int
    L._points_ready = True


def _points_lib():
    L = lib()
    _register_points(L)
    return L


def cost_points(X, Y, kind=SQEUCLID, cost_scale=1.0, split=0, out=None):
    """Cost matrix from point clouds X [n, d], Y [m, d] (float32, device); a batch
    X [B, n, d], Y [B, m, d] gives [B, n, m] in one call."""
    import torch
    if X.dim() == 3:
        _check_dev(X, torch.float32, "X", 3)
        _check_dev(Y, torch.float32, "Y", 3)
        X = X.contiguous()
        Y = Y.contiguous()
        B, n, d = X.shape
        m = Y.shape[1]
        if Y.shape[0] != B or Y.shape[2] != d:
            raise ValueError("X and Y must have the same batch and feature dimensions")
        if out is None:
            out = torch.empty((B, n, m), dtype=torch.float32, device=X.device)
        if out.shape != (B, n, m) or out.stride(2) != 1 or out.stride(0) != n * out.stride(1):
            raise ValueError("out must be a contiguous-row [B, n, m] tensor")
        st = _points_lib().accsk_cost_points_batched(_ptr(X), _ptr(Y), B, n, m, d, int(kind), float(cost_scale),
                                                     int(split), _ptr(out), out.stride(1), _stream_ptr())
        if st != OK:
            raise AccskError(st, "accsk_cost_points_batched")
        return out
    _check_dev(X, torch.float32, "X", 2)
    _check_dev(Y, torch.float32, "Y", 2)
    X = X.contiguous()
    Y = Y.contiguous()
    n, d = X.shape
    m = Y.shape[0]
    if Y.shape[1] != d:
        raise ValueError("X and Y must have the same feature dimension")
    if out is None:
        out = torch.empty((n, m), dtype=torch.float32, device=X.device)
    st = _points_lib().accsk_cost_points(_ptr(X), _ptr(Y), n, m, d, int(kind), float(cost_scale), int(split),
                                         _ptr(out), out.stride(0), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_cost_points")
    return out


def cost_max_points(X, Y, kind=SQEUCLID):
    """Exact maximum of the raw point-cloud cost (FP64 entries), as a Python float."""
    import torch
    _check_dev(X, torch.float32, "X", 2)
    _check_dev(Y, torch.float32, "Y", 2)
    X, Y = X.contiguous(), Y.contiguous()
    out = ctypes.c_double()
    st = _points_lib().accsk_cost_max_points(_ptr(X), _ptr(Y), X.shape[0], Y.shape[0], X.shape[1], int(kind),
                                             ctypes.byref(out), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_cost_max_points")
    return out.value


def plan_points(X, Y, f, g, eps, kind=SQEUCLID, cost_scale=1.0, row0=0, rows=None, out=None):
    """FP32 rows of the plan P_ij = exp((f_i + g_j - C_ij)/eps), C from the points in FP64."""
    import torch
    _check_dev(X, torch.float32, "X", 2)
    _check_dev(Y, torch.float32, "Y", 2)
    X, Y, f, g = X.contiguous(), Y.contiguous(), f.contiguous(), g.contiguous()
    n, d = X.shape
    m = Y.shape[0]
    rows = n - row0 if rows is None else rows
    if out is None:
        out = torch.empty((rows, m), dtype=torch.float32, device=X.device)
    st = _points_lib().accsk_plan_points(_ptr(X), _ptr(Y), n, m, d, int(kind), float(cost_scale), float(eps),
                                         _ptr(f), _ptr(g), int(row0), int(rows), _ptr(out), out.stride(0),
                                         _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_plan_points")
    return out


def barycentric_points(X, Y, f, g, eps, kind=SQEUCLID, cost_scale=1.0):
    """T_i = sum_j P_ij y_j / sum_j P_ij (float32 [n, d]), P recomputed on the device."""
    import torch
    _check_dev(X, torch.float32, "X", 2)
    _check_dev(Y, torch.float32, "Y", 2)
    X, Y, f, g = X.contiguous(), Y.contiguous(), f.contiguous(), g.contiguous()
    T = torch.empty_like(X)
    st = _points_lib().accsk_barycentric_points(_ptr(X), _ptr(Y), X.shape[0], Y.shape[0], X.shape[1], int(kind),
                                                float(cost_scale), float(eps), _ptr(f), _ptr(g), _ptr(T),
                                                _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_barycentric_points")
    return T


def topk_points(X, Y, f, g, eps, k=1, kind=SQEUCLID, cost_scale=1.0):
    """Row top-k of the plan: (int64 [n, k] column indices, float64 [n, k] plan values)."""
    import torch
    _check_dev(X, torch.float32, "X", 2)
    _check_dev(Y, torch.float32, "Y", 2)
    X, Y, f, g = X.contiguous(), Y.contiguous(), f.contiguous(), g.contiguous()
    n = X.shape[0]
    idx = torch.empty((n, k), dtype=torch.int64, device=X.device)
    val = torch.empty((n, k), dtype=torch.float64, device=X.device)
    st = _points_lib().accsk_topk_points(_ptr(X), _ptr(Y), n, Y.shape[0], X.shape[1], int(kind), float(cost_scale),
                                         float(eps), _ptr(f), _ptr(g), int(k), _ptr(idx), _ptr(val), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_topk_points")
    return idx, val


def _as_batched(X, Y, a, b):
    import torch
    single = X.dim() == 2
    if single:
        X, Y, a, b = X[None], Y[None], a[None], b[None]
    _check_dev(X, torch.float32, "X", 3)
    _check_dev(Y, torch.float32, "Y", 3)
    _check_dev(a, torch.float64, "a", 2)
    _check_dev(b, torch.float64, "b", 2)
    B, n, d = X.shape
    if Y.shape[0] != B or Y.shape[2] != d or a.shape != (B, n) or b.shape != (B, Y.shape[1]):
        raise ValueError("inconsistent point-cloud batch shapes")
    return single, X.contiguous(), Y.contiguous(), a.contiguous(), b.contiguous()


def solve_points(X, Y, a, b, eps, kind=SQEUCLID, cost_scale=1.0, split=0, tol=1e-6, method=ACC,
                 max_iter=100000, mu0=None, m0=None, w_rule=None, flags=0, on_the_fly=False, raise_on_error=True,
                 trace=False):
    """EOT between point clouds.  X [n,d] / [B,n,d] float32, a [n] / [B,n] float64.

    on_the_fly: form the cost in every step instead of storing it (d <= 16;
    implied for m > 8192).  Returns (f, g, results): f, g shaped like a, b;
    results a list of dicts.  trace=True (one problem only) adds results[0]["trace"],
    the L1 marginal error of every Sinkhorn step.
    """
    if on_the_fly:
        flags = int(flags) | FLAG_ON_THE_FLY
    import torch
    single, X, Y, a, b = _as_batched(X, Y, a, b)
    B, n, d = X.shape
    m = Y.shape[1]
    f = torch.empty((B, n), dtype=torch.float64, device=X.device)
    g = torch.empty((B, m), dtype=torch.float64, device=X.device)
    p = default_params(method=method, eps=float(eps), tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0,
                       w_rule=w_rule, split=int(split), flags=int(flags))
    tbuf = _trace_buffer(p, trace, max_iter, X.device)
    res = (Result * B)()
    st = _points_lib().accsk_solve_points_batched(_ptr(X), _ptr(Y), B, n, m, d, int(kind), float(cost_scale),
                                                  _ptr(a), _ptr(b), ctypes.byref(p), _ptr(f), _ptr(g), res,
                                                  _stream_ptr())
    if raise_on_error and st not in (OK, NOT_CONVERGED):
        raise AccskError(st, "accsk_solve_points_batched")
    out = [r.to_dict() for r in res]
    if tbuf is not None:
        out[0]["trace"] = tbuf[:max(0, min(res[0].sinkhorn_steps, tbuf.numel()))].cpu().numpy()
    if single:
        return f[0], g[0], out
    return f, g, out


def solve_points_async(X, Y, a, b, eps, kind=SQEUCLID, cost_scale=1.0, split=0, tol=1e-6, method=ACC,
                       max_iter=100000, mu0=None, m0=None, w_rule=None, flags=0, on_the_fly=False, rec=None):
    """Stream-ordered solve_points (batched shapes [B, n, d] or single [n, d]): returns (f, g, rec) at once."""
    if on_the_fly:
        flags = int(flags) | FLAG_ON_THE_FLY
    import torch
    single, X, Y, a, b = _as_batched(X, Y, a, b)
    B, n, d = X.shape
    m = Y.shape[1]
    f = torch.empty((B, n), dtype=torch.float64, device=X.device)
    g = torch.empty((B, m), dtype=torch.float64, device=X.device)
    if rec is None:
        rec = result_records(B, X.device)
    p = default_params(method=method, eps=float(eps), tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0,
                       w_rule=w_rule, split=int(split), flags=int(flags))
    st = _points_lib().accsk_solve_points_batched_async(_ptr(X), _ptr(Y), B, n, m, d, int(kind),
                                                        float(cost_scale), _ptr(a), _ptr(b), ctypes.byref(p),
                                                        _ptr(f), _ptr(g), _ptr(rec), _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_solve_points_batched_async")
    if single:
        return f[0], g[0], rec
    return f, g, rec


def backward_points(X, Y, a, b, f, g, eps, kind=SQEUCLID, cost_scale=1.0, grad_scale=None, marginals=True):
    """Envelope-theorem gradients of EOT at potentials (f, g).

    Returns (dX, dY, da, db) shaped like the inputs (da, db None if not asked).
    grad_scale: None or float64 device tensor [B] (or scalar tensor for one problem).
    """
    import torch
    single, X, Y, a, b = _as_batched(X, Y, a, b)
    B, n, d = X.shape
    m = Y.shape[1]
    f = f.reshape(B, n).contiguous()
    g = g.reshape(B, m).contiguous()
    _check_dev(f, torch.float64, "f")
    _check_dev(g, torch.float64, "g")
    dX = torch.empty_like(X)
    dY = torch.empty_like(Y)
    da = torch.empty_like(a) if marginals else None
    db = torch.empty_like(b) if marginals else None
    gs = None
    if grad_scale is not None:
        gs = grad_scale.to(device=X.device, dtype=torch.float64).reshape(B).contiguous()
    st = _points_lib().accsk_backward_points(
        _ptr(X), _ptr(Y), B, n, m, d, int(kind), float(cost_scale), float(eps), _ptr(a), _ptr(b), _ptr(f),
        _ptr(g), _ptr(gs) if gs is not None else None, _ptr(dX), _ptr(dY),
        _ptr(da) if da is not None else None, _ptr(db) if db is not None else None, _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_backward_points")
    if single:
        return dX[0], dY[0], (da[0] if marginals else None), (db[0] if marginals else None)
    return dX, dY, da, db


def backward_dense(C, a, b, f, g, eps, grad_scale=None, cost=True, marginals=True):
    """Envelope-theorem gradients of EOT on an explicit cost at potentials (f, g).

    Returns (dC, da, db): dC = grad_scale * P (float32 [n, m], None if cost=False),
    da, db the gradients with respect to the un-normalized marginals (float64, None
    if marginals=False).  grad_scale: None or a float64 device scalar tensor.
    """
    import torch
    _check_dev(C, torch.float32, "C", 2)
    _check_dev(f, torch.float64, "f", 1)
    _check_dev(g, torch.float64, "g", 1)
    if C.stride(1) != 1:
        raise ValueError("C must have unit column stride")
    n, m = C.shape
    a = a.contiguous()
    b = b.contiguous()
    dC = torch.empty((n, m), dtype=torch.float32, device=C.device) if cost else None
    da = torch.empty_like(a) if marginals else None
    db = torch.empty_like(b) if marginals else None
    gs = None
    if grad_scale is not None:
        gs = grad_scale.to(device=C.device, dtype=torch.float64).reshape(1).contiguous()
    st = _points_lib().accsk_backward_dense(
        _ptr(C), n, m, C.stride(0), float(eps), _ptr(a), _ptr(b), _ptr(f.contiguous()), _ptr(g.contiguous()),
        _ptr(gs) if gs is not None else None, _ptr(dC) if dC is not None else None, m,
        _ptr(da) if da is not None else None, _ptr(db) if db is not None else None, _stream_ptr())
    if st != OK:
        raise AccskError(st, "accsk_backward_dense")
    return dC, da, db


def _eot_dense_function():
    import torch

    class EOTDenseLoss(torch.autograd.Function):
        """EOT value of one explicit-cost problem, differentiable in C, a and b.

        Forward solves with the library and returns the FP64 EOT value; backward
        gives dEOT/dC = P (eq:P-from-dual) and the marginal gradients, scaled by
        the incoming gradient, from accsk_backward_dense.
        """

        @staticmethod
        def forward(ctx, C, a, b, eps, tol, method):
            f, g, res = solve_dense(C, a, b, eps, tol=tol, method=method)
            ctx.save_for_backward(C, a, b, f, g)
            ctx.eps = eps
            return torch.tensor(res["eot_value"], dtype=torch.float64, device=C.device)

        @staticmethod
        def backward(ctx, grad):
            C, a, b, f, g = ctx.saved_tensors
            dC, da, db = backward_dense(C, a, b, f, g, ctx.eps, grad_scale=grad.detach(),
                                        cost=ctx.needs_input_grad[0],
                                        marginals=ctx.needs_input_grad[1] or ctx.needs_input_grad[2])
            return dC, da, db, None, None, None

    return EOTDenseLoss


_EOT_DENSE = None


def eot_loss_dense(C, a, b, eps, tol=1e-6, method=ACC):
    """Differentiable EOT value (torch.autograd) of an explicit FP32 cost C [n, m]; see EOTDenseLoss."""
    global _EOT_DENSE
    if _EOT_DENSE is None:
        _EOT_DENSE = _eot_dense_function()
    return _EOT_DENSE.apply(C, a, b, eps, tol, method)


def _eot_function():
    import torch

    class EOTLoss(torch.autograd.Function):
        """EOT value of point-cloud problems, differentiable in X, Y, a, b.

        Forward solves with the library and returns the FP64 EOT values [B];
        backward applies the envelope-theorem gradients (dEOT/dC = P) scaled
        by the incoming gradient, all in the library's kernels.
        """

        @staticmethod
        def forward(ctx, X, Y, a, b, eps, kind, cost_scale, split, tol, method):
            f, g, res = solve_points(X, Y, a, b, eps, kind=kind, cost_scale=cost_scale, split=split, tol=tol,
                                     method=method)
            ctx.save_for_backward(X, Y, a, b, f, g)
            ctx.cfg = (eps, kind, cost_scale)
            vals = torch.tensor([r["eot_value"] for r in res], dtype=torch.float64, device=X.device)
            return vals[0] if X.dim() == 2 else vals

        @staticmethod
        def backward(ctx, grad):
            X, Y, a, b, f, g = ctx.saved_tensors
            eps, kind, cost_scale = ctx.cfg
            dX, dY, da, db = backward_points(X, Y, a, b, f, g, eps, kind=kind, cost_scale=cost_scale,
                                             grad_scale=grad.detach().to(torch.float64),
                                             marginals=ctx.needs_input_grad[2] or ctx.needs_input_grad[3])
            return dX, dY, da, db, None, None, None, None, None, None

    return EOTLoss


_EOT = None


def eot_loss(X, Y, a, b, eps, kind=SQEUCLID, cost_scale=1.0, split=0, tol=1e-6, method=ACC):
    """Differentiable EOT value (torch.autograd) between point clouds; see EOTLoss."""
    global _EOT
    if _EOT is None:
        _EOT = _eot_function()
    return _EOT.apply(X, Y, a, b, eps, kind, cost_scale, split, tol, method)


# ---------------------------------------------------------------------------
# Serving loop
# ---------------------------------------------------------------------------

class Request(ctypes.Structure):
    _fields_ = [("X", _vp), ("Y", _vp), ("n", _i64), ("m", _i64), ("d", _i64), ("kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cost_scale", _dbl), ("a", _vp), ("b", _vp), ("eps", _dbl),
                ("f_out", _vp), ("g_out", _vp)]


def _register_server(L):
    if getattr(L, "_server_ready", False):
        return
    L.accsk_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(Params),
                                      ctypes.POINTER(ctypes.c_void_p)]
    L.accsk_server_create.restype = ctypes.c_int
    L.accsk_server_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.accsk_server_submit.restype = ctypes.c_int
    L.accsk_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]
    L.accsk_server_poll.restype = ctypes.c_int
    L.accsk_server_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
    L.accsk_server_info.restype = ctypes.c_int
    L.accsk_server_admission.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
    L.accsk_server_admission.restype = ctypes.c_int
    L.accsk_server_destroy.argtypes = [_vp]
    L.accsk_server_destroy.restype = ctypes.c_int
    L.accsk_clock_seconds.argtypes = []
    L.accsk_clock_seconds.restype = ctypes.c_double
    L._server_ready = True


def clock_seconds():
    L = lib()
    _register_server(L)
    return L.accsk_clock_seconds()


class Server:
    """Persistent serving loop (continuous batching of point-cloud requests).

    submit() queues a request and returns a ticket; poll() returns None until
    the request is done, then (f, g, result dict, (t_submit, t_admit, t_done)).
    The request's tensors are kept alive here until it is done.
    """

    def __init__(self, hbm_budget=1 << 30, max_slots=0, method=ACC, tol=1e-6, max_iter=100000, mu0=None, m0=None,
                 w_rule=None, split=0, flags=0):
        L = lib()
        _register_server(L)
        self._L = L
        p = default_params(method=method, tol=float(tol), max_iter=int(max_iter), mu0=mu0, m0=m0, w_rule=w_rule,
                           split=int(split), flags=int(flags))
        h = ctypes.c_void_p()
        st = L.accsk_server_create(int(hbm_budget), int(max_slots), ctypes.byref(p), ctypes.byref(h))
        if st != OK:
            raise AccskError(st, "accsk_server_create")
        self._h = h
        self._live = {}

    def submit(self, X, Y, a, b, eps, kind=SQEUCLID, cost_scale=1.0, f_out=None, g_out=None):
        import torch
        _check_dev(X, torch.float32, "X", 2)
        _check_dev(Y, torch.float32, "Y", 2)
        _check_dev(a, torch.float64, "a", 1)
        _check_dev(b, torch.float64, "b", 1)
        X, Y, a, b = X.contiguous(), Y.contiguous(), a.contiguous(), b.contiguous()
        n, d = X.shape
        m = Y.shape[0]
        if Y.shape[1] != d or a.shape[0] != n or b.shape[0] != m:
            raise ValueError("inconsistent request shapes")
        f = torch.empty(n, dtype=torch.float64, device=X.device) if f_out is None else f_out
        g = torch.empty(m, dtype=torch.float64, device=X.device) if g_out is None else g_out
        _check_dev(f, torch.float64, "f_out", 1)
        _check_dev(g, torch.float64, "g_out", 1)
        if f.shape[0] != n or g.shape[0] != m or not (f.is_contiguous() and g.is_contiguous()):
            raise ValueError("f_out / g_out must be contiguous [n] / [m]")
        req = Request(X.data_ptr(), Y.data_ptr(), n, m, d, int(kind), 0, float(cost_scale), a.data_ptr(),
                      b.data_ptr(), float(eps), f.data_ptr(), g.data_ptr())
        t = ctypes.c_uint64()
        st = self._L.accsk_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != OK:
            raise AccskError(st, "accsk_server_submit")
        self._live[t.value] = (X, Y, a, b, f, g)
        return t.value

    def poll(self, ticket):
        r = Result()
        done = ctypes.c_int()
        times = (ctypes.c_double * 3)()
        st = self._L.accsk_server_poll(self._h, ticket, ctypes.byref(r), ctypes.byref(done), times)
        if st != OK:
            raise AccskError(st, "accsk_server_poll")
        if not done.value:
            return None
        X, Y, a, b, f, g = self._live.pop(ticket)
        return f, g, r.to_dict(), (times[0], times[1], times[2])

    def wait(self, ticket, timeout=60.0):
        import time
        t0 = time.monotonic()
        while True:
            out = self.poll(ticket)
            if out is not None:
                return out
            if time.monotonic() - t0 > timeout:
                raise TimeoutError("request %d not done after %.1f s" % (ticket, timeout))
            time.sleep(20e-6)

    def info(self):
        v = (ctypes.c_int64 * 5)()
        st = self._L.accsk_server_info(self._h, v)
        if st != OK:
            raise AccskError(st, "accsk_server_info")
        return dict(workers=v[0], waiting=v[1], in_flight=v[2], launches=v[3], free_bytes=v[4])

    def admission(self):
        """Admission-by-footprint counters (see accsk_server_admission)."""
        v = (ctypes.c_int64 * 6)()
        st = self._L.accsk_server_admission(self._h, v)
        if st != OK:
            raise AccskError(st, "accsk_server_admission")
        return dict(space_waited=v[0], fit_failures=v[1], overtakes=v[2], peak_bytes_in_use=v[3],
                    peak_in_flight=v[4], budget=v[5])

    def close(self):
        if getattr(self, "_h", None):
            st = self._L.accsk_server_destroy(self._h)
            self._h = None
            self._live.clear()
            if st != OK:
                raise AccskError(st, "accsk_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
