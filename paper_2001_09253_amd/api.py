"""Thin Python binding of the C ABI in include/spline_solve.h.

Each function has the name of the C entry point it calls and only marshals
arguments (tensor/array -> pointer, size checks, error code -> exception);
every step of the spline path runs in the HIP library.  Device arguments are
torch CUDA tensors (float64 / int32 / int64, contiguous); host arguments of the
request API may be NumPy arrays or CPU tensors.  ``stream`` defaults to torch's
current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native
from ._native import SolveConfig, Tuning

OK, E_ARG, E_SIZE, E_ORDER, E_BUDGET, E_DEVICE, E_TICKET, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
PENDING, DONE, ERROR = 0, 1, 2
FP64, FP32_REFINE = 0, 1
PLAIN, NO_GRAPH = 1, 2
MAX_N_BLOCK = 16384
MAX_N_BATCH = 2048
MAX_N_SOLVE = 1 << 30
NOALLOC_SCRATCH_BYTES = 8 << 20

_NAMES = {OK: "OK", E_ARG: "E_ARG", E_SIZE: "E_SIZE", E_ORDER: "E_ORDER", E_BUDGET: "E_BUDGET",
          E_DEVICE: "E_DEVICE", E_TICKET: "E_TICKET", E_STATE: "E_STATE"}


class SolveError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__("%s failed: %s (%d)" % (what, _NAMES.get(code, "?"), code))
        self.code = code


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise SolveError(rc, what)


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dev(t, dtype=torch.float64, name="tensor", numel=None, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s needs at least %d elements" % (name, numel))
    return C.c_void_p(t.data_ptr())


def _any(a, name="array", optional=False):
    """Pointer of a host array/tensor or a device tensor (request API)."""
    if a is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous() or a.dtype != torch.float64:
            raise TypeError("%s must be a contiguous float64 tensor" % name)
        return C.c_void_p(a.data_ptr())
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("%s must be a C-contiguous float64 array" % name)
        return C.c_void_p(a.ctypes.data)
    raise TypeError("%s must be a NumPy array or a torch tensor" % name)


# -- device-level operations -------------------------------------------------------------

def spline_build(x, y, start_deriv, end_deriv, ypp, status=None, stream=None):
    n = x.numel()
    _check(_native.lib().spline_build(_dev(x, name="x"), _dev(y, name="y", numel=n), n, float(start_deriv),
                                      float(end_deriv), _dev(ypp, name="ypp", numel=n),
                                      _dev(status, torch.int32, "status", 1, optional=True), _stream(stream)),
           "spline_build")


def spline_solve_uniform(x, y, start_deriv, end_deriv, m, yq, ypp=None, status=None, stream=None):
    """Build and evaluate one curve in a single launch (status, if given, is
    set to E_ORDER on unordered knots and left as is otherwise)."""
    n = x.numel()
    _check(_native.lib().spline_solve_uniform(_dev(x, name="x"), _dev(y, name="y", numel=n), n, float(start_deriv),
                                              float(end_deriv), int(m), _dev(yq, name="yq", numel=int(m)),
                                              _dev(ypp, name="ypp", numel=n, optional=True),
                                              _dev(status, torch.int32, "status", 1, optional=True),
                                              _stream(stream)),
           "spline_solve_uniform")


def spline_solve_uniform_indexed(x, y, start_deriv, end_deriv, m, yq, idx, ypp=None, status=None, stream=None):
    """spline_solve_uniform that also writes every query's interval into idx
    (int32, m)."""
    n = x.numel()
    _check(_native.lib().spline_solve_uniform_indexed(
        _dev(x, name="x"), _dev(y, name="y", numel=n), n, float(start_deriv), float(end_deriv), int(m),
        _dev(yq, name="yq", numel=int(m)), _dev(ypp, name="ypp", numel=n, optional=True),
        _dev(idx, torch.int32, "idx", int(m)), _dev(status, torch.int32, "status", 1, optional=True),
        _stream(stream)), "spline_solve_uniform_indexed")


# evaluation formulas of spline_solve_uniform_variant (the paper's
# "Curve Interpolation" benchmark variants)
NEWINT_HOISTED = 0
NEWINT_ORIG = 1
NEWINT_NOINV = 2
SPLINT_DIV = 3
SPLINT_MUL = 4
HORNER = 5  # not one of the paper's variants
VARIANTS = {"newint": NEWINT_HOISTED, "newint__orig": NEWINT_ORIG, "newint__noinv": NEWINT_NOINV,
            "splint_one__div": SPLINT_DIV, "splint_one__mul": SPLINT_MUL, "horner": HORNER}


def spline_solve_uniform_variant(x, y, start_deriv, end_deriv, m, variant, yq, ypp=None, status=None, stream=None):
    """spline_solve_uniform on the wavefront-per-block kernel with the
    evaluation formula `variant` (a VARIANTS value)."""
    n = x.numel()
    _check(_native.lib().spline_solve_uniform_variant(
        _dev(x, name="x"), _dev(y, name="y", numel=n), n, float(start_deriv), float(end_deriv), int(m),
        int(variant), _dev(yq, name="yq", numel=int(m)), _dev(ypp, name="ypp", numel=n, optional=True),
        _dev(status, torch.int32, "status", 1, optional=True), _stream(stream)),
        "spline_solve_uniform_variant")


def spline_eval_uniform(x, y, ypp, m, yq, stream=None):
    n = x.numel()
    _check(_native.lib().spline_eval_uniform(_dev(x, name="x"), _dev(y, name="y", numel=n),
                                             _dev(ypp, name="ypp", numel=n), n, int(m),
                                             _dev(yq, name="yq", numel=int(m)), _stream(stream)),
           "spline_eval_uniform")


def spline_bracket_uniform(x, m, idx, stream=None):
    _check(_native.lib().spline_bracket_uniform(_dev(x, name="x"), x.numel(), int(m),
                                                _dev(idx, torch.int32, "idx", int(m)), _stream(stream)),
           "spline_bracket_uniform")


def spline_noop_uniform(x, m, out, stream=None):
    _check(_native.lib().spline_noop_uniform(_dev(x, name="x"), x.numel(), int(m),
                                             _dev(out, name="out", numel=int(m)), _stream(stream)),
           "spline_noop_uniform")


def spline_eval_points(x, y, ypp, xq, yq, d1=None, d2=None, idx=None, stream=None):
    n, m = x.numel(), xq.numel()
    _check(_native.lib().spline_eval_points(_dev(x, name="x"), _dev(y, name="y", numel=n),
                                            _dev(ypp, name="ypp", numel=n), n, _dev(xq, name="xq"), m,
                                            _dev(yq, name="yq", numel=m), _dev(d1, name="d1", numel=m, optional=True),
                                            _dev(d2, name="d2", numel=m, optional=True),
                                            _dev(idx, torch.int32, "idx", m, optional=True), _stream(stream)),
           "spline_eval_points")


def spline_pack_knots(x, y, ypp, packed, stream=None):
    """Interleave x, y, y'' of one curve into packed (3 n device doubles)."""
    n = x.numel()
    _check(_native.lib().spline_pack_knots(_dev(x, name="x"), _dev(y, name="y", numel=n),
                                           _dev(ypp, name="ypp", numel=n), n, _dev(packed, name="packed", numel=3 * n),
                                           _stream(stream)), "spline_pack_knots")


def spline_eval_points_packed(packed, xq, yq, d1=None, d2=None, idx=None, stream=None):
    """spline_eval_points on a curve packed by spline_pack_knots."""
    n, m = packed.numel() // 3, xq.numel()
    _check(_native.lib().spline_eval_points_packed(_dev(packed, name="packed"), n, _dev(xq, name="xq"), m,
                                                   _dev(yq, name="yq", numel=m),
                                                   _dev(d1, name="d1", numel=m, optional=True),
                                                   _dev(d2, name="d2", numel=m, optional=True),
                                                   _dev(idx, torch.int32, "idx", m, optional=True), _stream(stream)),
           "spline_eval_points_packed")


def spline_batch_eval_points(koff, qoff, x, y, ypp, xq, yq, d1=None, d2=None, idx=None, stream=None):
    """Explicit points of many curves in one launch: koff, qoff device int64
    (count + 1, CSR), x, y, ypp per knot, xq and yq (and d1, d2, idx) per
    query, as many as xq holds."""
    count = koff.numel() - 1
    m = xq.numel()
    _check(_native.lib().spline_batch_eval_points(
        count, m, _dev(koff, torch.int64, "koff"), _dev(qoff, torch.int64, "qoff", count + 1), _dev(x, name="x"),
        _dev(y, name="y", numel=x.numel()), _dev(ypp, name="ypp", numel=x.numel()), _dev(xq, name="xq"),
        _dev(yq, name="yq", numel=m), _dev(d1, name="d1", numel=m, optional=True),
        _dev(d2, name="d2", numel=m, optional=True), _dev(idx, torch.int32, "idx", m, optional=True),
        _stream(stream)), "spline_batch_eval_points")


# -- batched plans --------------------------------------------------------------------------

class Plan:
    """Owning wrapper of a spline_plan handle."""

    def __init__(self, handle, count, koff, qoff):
        self.handle = handle
        self.count = count
        self.koff = koff
        self.qoff = qoff

    def __del__(self):
        self.destroy()

    def destroy(self):
        if getattr(self, "handle", None):
            _native.lib().spline_plan_destroy(self.handle)
            self.handle = None


def spline_plan_create(koff, qoff, precision=FP64, tuning=None, device=None):
    """qoff None: a build-only plan (y'' of every curve, no queries)."""
    koff = np.ascontiguousarray(koff, dtype=np.int64)
    qoff = None if qoff is None else np.ascontiguousarray(qoff, dtype=np.int64)
    count = len(koff) - 1
    dev = torch.cuda.current_device() if device is None else int(device)
    h = C.c_void_p()
    t = C.byref(tuning) if tuning is not None else None
    _check(_native.lib().spline_plan_create(dev, count, koff.ctypes.data_as(C.c_void_p),
                                            None if qoff is None else qoff.ctypes.data_as(C.c_void_p),
                                            int(precision), t, C.byref(h)),
           "spline_plan_create")
    return Plan(h, count, koff, qoff)


def _plan_args(plan, b):
    n_tot = int(plan.koff[-1])
    build_only = plan.qoff is None
    m_tot = 0 if build_only else int(plan.qoff[-1])
    return [_dev(b["x"], name="x", numel=n_tot), _dev(b["y"], name="y", numel=n_tot),
            _dev(b["sd"], name="sd", numel=plan.count), _dev(b["ed"], name="ed", numel=plan.count),
            _dev(b["koff"], torch.int64, "koff", plan.count + 1),
            _dev(b.get("qoff"), torch.int64, "qoff", plan.count + 1, optional=build_only),
            _dev(b.get("yq"), name="yq", numel=m_tot, optional=build_only), _dev(b["ypp"], name="ypp", numel=n_tot)]


def spline_plan_run(plan, bufs, status=None, stream=None):
    """bufs: dict of device tensors x, y, sd, ed, koff, qoff, yq, ypp."""
    _check(_native.lib().spline_plan_run(plan.handle, *_plan_args(plan, bufs),
                                         _dev(status, torch.int32, "status", plan.count, optional=True),
                                         _stream(stream)), "spline_plan_run")


def spline_plan_run_indexed(plan, bufs, idx, status=None, stream=None):
    """spline_plan_run that also writes every query's interval (within its
    curve) into idx (int32, sum m)."""
    _check(_native.lib().spline_plan_run_indexed(plan.handle, *_plan_args(plan, bufs),
                                                 _dev(idx, torch.int32, "idx",
                                                      0 if plan.qoff is None else int(plan.qoff[-1])),
                                                 _dev(status, torch.int32, "status", plan.count, optional=True),
                                                 _stream(stream)), "spline_plan_run_indexed")


def spline_plan_capture(plan, bufs, status=None, stream=None):
    _check(_native.lib().spline_plan_capture(plan.handle, *_plan_args(plan, bufs),
                                             _dev(status, torch.int32, "status", plan.count, optional=True),
                                             _stream(stream)), "spline_plan_capture")


def spline_plan_replay(plan, stream=None):
    _check(_native.lib().spline_plan_replay(plan.handle, _stream(stream)), "spline_plan_replay")


def spline_plan_autotune(plan, bufs, reps=10, cache_path=None):
    best = Tuning()
    ms = C.c_double()
    _check(_native.lib().spline_plan_autotune(plan.handle, *_plan_args(plan, bufs), int(reps),
                                              cache_path.encode() if cache_path else None, C.byref(best),
                                              C.byref(ms)), "spline_plan_autotune")
    return best, ms.value


WAVE_ITEM_DTYPE = np.dtype([("ko", "<i8"), ("qo", "<i8"), ("m", "<i8"), ("inst", "<i4"), ("n", "<i4"),
                            ("j0", "<i2"), ("j1", "<i2"), ("s", "<i4"), ("S", "<i4"), ("pad", "<i4")])


def spline_plan_get_tables(plan):
    """(work items as a structured array, curves of the first launch,
    rows of the widest span a wavefront holds)."""
    ni, nl, rows = C.c_int64(), C.c_int64(), C.c_int64()
    L = _native.lib()
    _check(L.spline_plan_get_tables(plan.handle, None, 0, C.byref(ni), C.byref(nl), C.byref(rows)),
           "spline_plan_get_tables")
    off = (ni.value * WAVE_ITEM_DTYPE.itemsize + 255) & ~255
    buf = np.zeros(off + 4 * nl.value + 16, dtype=np.uint8)
    _check(L.spline_plan_get_tables(plan.handle, C.c_void_p(buf.ctypes.data), buf.nbytes, C.byref(ni), C.byref(nl),
                                    C.byref(rows)), "spline_plan_get_tables")
    items = buf[:ni.value * WAVE_ITEM_DTYPE.itemsize].view(WAVE_ITEM_DTYPE).copy()
    lane = buf[off:off + 4 * nl.value].view(np.int32).copy()
    return items, lane, rows.value


def spline_plan_get_tuning(plan):
    t = Tuning()
    _check(_native.lib().spline_plan_get_tuning(plan.handle, C.byref(t)), "spline_plan_get_tuning")
    return t


def spline_batch_run_noalloc(koff, qoff, bufs, precision=FP64, tuning=None, status=None, stream=None):
    """spline_plan_create + spline_plan_run without device allocation (the
    tables go to the library's fixed device buffer).  koff/qoff: host int64
    offsets; bufs as for spline_plan_run (device tensors, including the same
    offsets on the device)."""
    koff = np.ascontiguousarray(koff, dtype=np.int64)
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    count = len(koff) - 1
    n_tot, m_tot = int(koff[-1]), int(qoff[-1])
    args = [_dev(bufs["x"], name="x", numel=n_tot), _dev(bufs["y"], name="y", numel=n_tot),
            _dev(bufs["sd"], name="sd", numel=count), _dev(bufs["ed"], name="ed", numel=count),
            _dev(bufs["koff"], torch.int64, "koff", count + 1), _dev(bufs["qoff"], torch.int64, "qoff", count + 1),
            _dev(bufs["yq"], name="yq", numel=m_tot), _dev(bufs["ypp"], name="ypp", numel=n_tot)]
    _check(_native.lib().spline_batch_run_noalloc(count, koff.ctypes.data_as(C.c_void_p),
                                                  qoff.ctypes.data_as(C.c_void_p), int(precision),
                                                  C.byref(tuning) if tuning is not None else None, *args,
                                                  _dev(status, torch.int32, "status", count, optional=True),
                                                  _stream(stream)), "spline_batch_run_noalloc")


# -- request API ------------------------------------------------------------------------------

def solve_create(device=0, hbm_budget_bytes=200 << 30, max_slots=65536, precision=FP64, flags=0,
                 max_inflight=2, stream=None):
    cfg = SolveConfig(int(device), int(hbm_budget_bytes), int(max_slots), int(precision), int(flags),
                      int(max_inflight), None if stream is None else _stream(stream))
    h = C.c_void_p()
    _check(_native.lib().solve_create(C.byref(cfg), C.byref(h)), "solve_create")
    return h


def solve_submit(ctx, knots, values, start_deriv, end_deriv, xq, m, yq_out, ypp_out=None):
    """Returns the ticket.  yq_out / ypp_out must stay alive until the ticket is
    reported DONE or ERROR."""
    n = int(len(knots))
    if len(values) != n:
        raise SolveError(E_SIZE, "solve_submit")
    t = C.c_uint64()
    _check(_native.lib().solve_submit(ctx, _any(knots, "knots"), _any(values, "values"), n, float(start_deriv),
                                      float(end_deriv), _any(xq, "xq", optional=True), int(m),
                                      _any(yq_out, "yq_out"), _any(ypp_out, "ypp_out", optional=True),
                                      C.byref(t)), "solve_submit")
    return t.value


def solve_poll(ctx, ticket):
    st = C.c_int()
    _check(_native.lib().solve_poll(ctx, int(ticket), C.byref(st)), "solve_poll")
    return st.value


def solve_wait(ctx, ticket, timeout_ms=-1):
    st = C.c_int()
    _check(_native.lib().solve_wait(ctx, int(ticket), C.byref(st), int(timeout_ms)), "solve_wait")
    return st.value


def solve_ticket_info(ctx, ticket):
    t = (C.c_double * 4)()
    code = C.c_int()
    _check(_native.lib().solve_ticket_info(ctx, int(ticket), t, C.byref(code)), "solve_ticket_info")
    return list(t), code.value


def solve_clock():
    return _native.lib().solve_clock()


def solve_stats(ctx):
    out = (C.c_uint64 * 8)()
    _check(_native.lib().solve_stats(ctx, out), "solve_stats")
    keys = ["submitted", "completed", "failed", "batches", "resident_bytes", "peak_resident_bytes",
            "waiting", "peak_batch"]
    return dict(zip(keys, list(out)))


def solve_memory(ctx):
    out = (C.c_uint64 * 2)()
    _check(_native.lib().solve_memory(ctx, out), "solve_memory")
    return {"device_bytes": int(out[0]), "peak_device_bytes": int(out[1])}


def solve_inject_fault(ctx):
    _check(_native.lib().solve_inject_fault(ctx), "solve_inject_fault")


def solve_destroy(ctx):
    _check(_native.lib().solve_destroy(ctx), "solve_destroy")


def spline_plan_destroy(plan):
    """Release a plan (also done when the Plan object is collected)."""
    plan.destroy()
