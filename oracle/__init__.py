"""FP64 CPU oracle for the cubic-spline hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

The arithmetic lives in ``spline_oracle.c`` (plain C, FP64, no contraction);
this module compiles it with gcc on first use and marshals NumPy arrays
through ctypes.  Every function follows a passage of the paper, cited in the C
source: the row equations of "Generating Second Derivatives" and "Start and
End Derivatives", a banded Gaussian elimination with partial pivoting, binary
search bracketing and the A, B, C, D interpolation formula of "Fast
Interpolation".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spline_oracle.c")
LIB = os.path.join(HERE, "liboracle_spline.so")

OK, E_ARG, E_SIZE, E_ORDER, E_SINGULAR, E_NOMEM = 0, -1, -2, -3, -8, -9

_lock = threading.Lock()
_lib = None

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_i32 = C.POINTER(C.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle into a shared library next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-D_POSIX_C_SOURCE=200809L", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            sig = {
                "oracle_validate": (C.c_int, [_d, C.c_int64]),
                "oracle_rows": (C.c_int, [_d, _d, C.c_int64, C.c_double, C.c_double, _d, _d, _d, _d]),
                "oracle_band_solve": (C.c_int, [C.c_int64, _d, _d, _d, _d, _d]),
                "oracle_second_derivatives": (C.c_int, [_d, _d, C.c_int64, C.c_double, C.c_double, _d]),
                "oracle_uniform_query": (C.c_double, [C.c_double, C.c_double, C.c_int64, C.c_int64]),
                "oracle_uniform_queries": (None, [C.c_double, C.c_double, C.c_int64, _d]),
                "oracle_bracket": (C.c_int64, [_d, C.c_int64, C.c_double]),
                "oracle_eval_points": (C.c_int, [_d, _d, _d, C.c_int64, _d, C.c_int64, _d, _i64]),
                "oracle_eval_points_derivs": (C.c_int, [_d, _d, _d, C.c_int64, _d, C.c_int64, _d, _d]),
                "oracle_bracket_uniform": (C.c_int, [_d, C.c_int64, C.c_int64, _i64]),
                "oracle_spline_uniform": (C.c_int, [_d, _d, C.c_int64, C.c_double, C.c_double,
                                                    C.c_int64, _d, _d]),
                "oracle_uniform_range": (C.c_int, [_d, _d, _d, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                                   _d, _i64, C.c_int]),
                "oracle_spline_uniform_sample": (C.c_int, [_d, _d, C.c_int64, C.c_double, C.c_double,
                                                           C.c_int64, _i64, C.c_int64, _d, _d]),
                "oracle_batch_uniform": (C.c_int, [C.c_int64, _i64, _i64, _d, _d, _d, _d, _d, _d,
                                                   _i32, C.c_int]),
                "oracle_eval_interval": (C.c_double, [_d, _d, _d, C.c_int64, C.c_double]),
                "oracle_eval_derivs": (None, [_d, _d, _d, C.c_int64, C.c_double, _d, _d]),
                "oracle_now": (C.c_double, []),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error code %d" % code)
        self.code = code


def _p(a, t=_d):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc != OK:
        raise OracleError(rc)


def validate(x) -> int:
    x = _f64(x)
    return lib().oracle_validate(_p(x), len(x))


def rows(x, y, start_deriv, end_deriv):
    """(lo, di, up, rhs) of the tridiagonal system for y''."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    out = [np.zeros(n) for _ in range(4)]
    _check(lib().oracle_rows(_p(x), _p(y), n, float(start_deriv), float(end_deriv), *[_p(a) for a in out]))
    return tuple(out)


def band_solve(lo, di, up, rhs):
    lo, di, up, rhs = (_f64(a) for a in (lo, di, up, rhs))
    out = np.zeros(len(di))
    _check(lib().oracle_band_solve(len(di), _p(lo), _p(di), _p(up), _p(rhs), _p(out)))
    return out


def second_derivatives(x, y, start_deriv, end_deriv):
    x, y = _f64(x), _f64(y)
    out = np.zeros(len(x))
    _check(lib().oracle_second_derivatives(_p(x), _p(y), len(x), float(start_deriv),
                                           float(end_deriv), _p(out)))
    return out


def uniform_query(x0, xlast, m, k):
    """Position of uniform query k of m (one query)."""
    return float(lib().oracle_uniform_query(float(x0), float(xlast), int(m), int(k)))


def uniform_queries(x0, xlast, m):
    q = np.zeros(int(m))
    lib().oracle_uniform_queries(float(x0), float(xlast), int(m), _p(q))
    return q


def bracket(x, q):
    x = _f64(x)
    return int(lib().oracle_bracket(_p(x), len(x), float(q)))


def bracket_uniform(x, m):
    x = _f64(x)
    idx = np.zeros(int(m), dtype=np.int64)
    _check(lib().oracle_bracket_uniform(_p(x), len(x), int(m), _p(idx, _i64)))
    return idx


def eval_points(x, y, ypp, q, with_index=False):
    x, y, ypp, q = _f64(x), _f64(y), _f64(ypp), _f64(q)
    out = np.zeros(len(q))
    idx = np.zeros(len(q), dtype=np.int64)
    _check(lib().oracle_eval_points(_p(x), _p(y), _p(ypp), len(x), _p(q), len(q), _p(out), _p(idx, _i64)))
    return (out, idx) if with_index else out


def eval_on_interval(x, y, ypp, i, q):
    """(value, first derivative, second derivative) of interval i's cubic at q."""
    x, y, ypp = _f64(x), _f64(y), _f64(ypp)
    d1 = C.c_double()
    d2 = C.c_double()
    v = lib().oracle_eval_interval(_p(x), _p(y), _p(ypp), int(i), float(q))
    lib().oracle_eval_derivs(_p(x), _p(y), _p(ypp), int(i), float(q), C.byref(d1), C.byref(d2))
    return v, d1.value, d2.value


def eval_points_derivs(x, y, ypp, q):
    x, y, ypp, q = _f64(x), _f64(y), _f64(ypp), _f64(q)
    d1 = np.zeros(len(q))
    d2 = np.zeros(len(q))
    _check(lib().oracle_eval_points_derivs(_p(x), _p(y), _p(ypp), len(x), _p(q), len(q), _p(d1), _p(d2)))
    return d1, d2


def spline_uniform(x, y, start_deriv, end_deriv, m):
    """(yq[m], ypp[n]) for m uniform queries between the first and last knot."""
    x, y = _f64(x), _f64(y)
    yq = np.zeros(int(m))
    ypp = np.zeros(len(x))
    _check(lib().oracle_spline_uniform(_p(x), _p(y), len(x), float(start_deriv), float(end_deriv),
                                       int(m), _p(yq), _p(ypp)))
    return yq, ypp


def uniform_range(x, y, ypp, m, k0, k1, threads: int = 0):
    """(values, intervals) of uniform queries k0..k1-1 of m, given ypp[n]."""
    x, y, ypp = _f64(x), _f64(y), _f64(ypp)
    cnt = int(k1) - int(k0)
    yq = np.zeros(max(cnt, 0))
    idx = np.zeros(max(cnt, 0), dtype=np.int64)
    _check(lib().oracle_uniform_range(_p(x), _p(y), _p(ypp), len(x), int(m), int(k0), int(k1), _p(yq),
                                      _p(idx, _i64), int(threads)))
    return yq, idx


def spline_uniform_sample(x, y, start_deriv, end_deriv, m, ks):
    """Values at the uniform query indices ks only, plus ypp[n]."""
    x, y = _f64(x), _f64(y)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    yq = np.zeros(len(ks))
    ypp = np.zeros(len(x))
    _check(lib().oracle_spline_uniform_sample(_p(x), _p(y), len(x), float(start_deriv), float(end_deriv),
                                              int(m), _p(ks, _i64), len(ks), _p(yq), _p(ypp)))
    return yq, ypp


def batch_uniform(koff, qoff, x, y, sd, ed, threads: int = 0):
    """CSR batch; returns (yq, ypp, status, threads_used)."""
    koff = np.ascontiguousarray(koff, dtype=np.int64)
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    x, y, sd, ed = _f64(x), _f64(y), _f64(sd), _f64(ed)
    count = len(koff) - 1
    yq = np.zeros(int(qoff[-1]))
    ypp = np.zeros(int(koff[-1]))
    st = np.zeros(count, dtype=np.int32)
    used = lib().oracle_batch_uniform(count, _p(koff, _i64), _p(qoff, _i64), _p(x), _p(y), _p(sd), _p(ed),
                                      _p(yq), _p(ypp), _p(st, _i32), int(threads))
    return yq, ypp, st, used


def now() -> float:
    return lib().oracle_now()
