"""Planted mistakes in the oracle must fail its pins.

Each mutation edits a copy of oracle/spline_oracle.c (on the CPU, in a temporary
directory), compiles it, and runs a compact battery of the pins of
test_oracle_pins.py against it: the paper's Table 1 values, the exact rational
spline for every end condition, the scan-based bracketing, a dense solve with
row swaps, and the strict natural sentinel.  The unmutated source must pass the
same battery.  This shows that a dropped term, a wrong sign, a wrong index, a
transposed operand or an off-by-one in the oracle would not go unnoticed.
"""
import ctypes as C
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_spline import ExactSpline
from paper_2001_09253_amd import workloads as w

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)

MUTATIONS = {
    "end_row_prose_order": ("lo[n - 1] = h;\n        di[n - 1] = 2.0 * h;",
                            "lo[n - 1] = 2.0 * h;\n        di[n - 1] = h;"),
    "dropped_factor_2": ("di[j] = 2.0 * (x[j + 1] - x[j - 1]);", "di[j] = (x[j + 1] - x[j - 1]);"),
    "start_slope_sign": ("rhs[0] = 6.0 * ((y[1] - y[0]) / h - start_deriv);",
                         "rhs[0] = 6.0 * ((y[1] - y[0]) / h + start_deriv);"),
    "wrong_index_up": ("up[j] = x[j + 1] - x[j];", "up[j] = x[j] - x[j - 1];"),
    "bracket_tie": ("if (x[mid] < q) lo = mid + 1;", "if (x[mid] <= q) lo = mid + 1;"),
    "eval_transposed": ("return A * y[i] + B * y[i + 1]", "return B * y[i] + A * y[i + 1]"),
    "elim_sign": ("r[k + 1] -= l * r[k];", "r[k + 1] += l * r[k];"),
    "backsub_drop_fill": ("out[k] = (r[k] - f1[k] * out[k + 1] - f2[k] * out[k + 2]) / dg[k];",
                          "out[k] = (r[k] - f1[k] * out[k + 1]) / dg[k];"),
    "query_fused": ("double step = (double)k * h;\n    return x0 + step;", "return fma((double)k, h, x0);"),
    "query_step": ("double h = (xlast - x0) / (double)(m - 1);", "double h = (xlast - x0) / (double)m;"),
    "sentinel_not_strict": ("return deriv > 0.99e30;", "return deriv >= 0.99e30;"),
    "eval_C_factor": ("double C = (A * A * A - A) * (h * h) / 6.0;", "double C = (A * A * A - A) * (h * h) / 3.0;"),
    "rhs_dropped_term": ("rhs[j] = 6.0 * ((y[j + 1] - y[j]) / (x[j + 1] - x[j]) - (y[j] - y[j - 1]) / (x[j] - x[j - 1]));",
                         "rhs[j] = 6.0 * ((y[j + 1] - y[j]) / (x[j + 1] - x[j]));"),
}


def _compile(src_text, tag):
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    src = os.path.join(d, "m.c")
    so = os.path.join(d, "lib%s.so" % tag)
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-D_POSIX_C_SOURCE=200809L",
                    "-shared", "-fPIC", src, "-o", so, "-lm"], check=True)
    L = C.CDLL(so)
    L.oracle_spline_uniform.argtypes = [_d, _d, C.c_int64, C.c_double, C.c_double, C.c_int64, _d, _d]
    L.oracle_bracket_uniform.argtypes = [_d, C.c_int64, C.c_int64, _i64]
    L.oracle_band_solve.argtypes = [C.c_int64, _d, _d, _d, _d, _d]
    L.oracle_uniform_queries.argtypes = [C.c_double, C.c_double, C.c_int64, _d]
    L.oracle_uniform_queries.restype = None
    return L


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _battery(L):
    """Returns the list of pins the library fails."""
    failed = []

    def spline(x, y, sd, ed, m):
        yq = np.zeros(m)
        ypp = np.zeros(len(x))
        rc = L.oracle_spline_uniform(_p(x), _p(y), len(x), sd, ed, m, _p(yq), _p(ypp))
        return rc, yq, ypp

    # Table 1
    printed = np.array([0, 306.924794, -1213.299177, 2450.276370, -679.188305, 310.152841, -80.047486,
                        12.113742, -5.706845, 0.029250, -1.048158, -1.612180, 0])
    rc, _, ypp = spline(w.HAND_KNOTS, w.HAND_VALUES, 1e32, 1e32, 16)
    if rc or np.max(np.abs(ypp - printed)) > 5e-7 + 1e-12:
        failed.append("table1")
    # exact rational spline, every end condition
    for seed, (sd, ed) in enumerate([(1e32, 1e32), (0.0, 0.0), (-1.0, 1.0), (1e32, 0.5), (-2.0, 1e32)]):
        x, y = w.paper_curve(np.random.default_rng(seed), 6)
        ex = ExactSpline(x, y, sd, ed)
        m = 23
        rc, yq, ypp = spline(x, y, sd, ed, m)
        q = oracle.uniform_queries(x[0], x[-1], m)
        t_ypp = np.array([float(v) for v in ex.second_derivatives()])
        t_yq = np.array([float(ex.value(Fraction(float(v)))) for v in q])
        s = np.max(np.abs(t_ypp)) + 1.0
        if rc or np.max(np.abs(ypp - t_ypp)) > 1e-12 * s or np.max(np.abs(yq - t_yq)) > 1e-12 * s:
            failed.append("exact:%d" % seed)
    # uniform queries: the bits of np.linspace, the paper's sampling call
    for x0, x1, m in ((0.0, 1.0, 11), (0.1, 1e6, 100003), (-7.5, -0.25, 65537)):
        q = np.zeros(m)
        L.oracle_uniform_queries(x0, x1, m, _p(q))
        if not np.array_equal(q, np.linspace(x0, x1, m)):
            failed.append("queries")
            break
    # bracketing against the paper's scan loop, queries placed on the knots
    x = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    idx = np.zeros(9, dtype=np.int64)
    L.oracle_bracket_uniform(_p(x), 5, 9, _p(idx, _i64))
    if list(idx) != [0, 0, 0, 1, 1, 2, 2, 3, 3]:
        failed.append("bracket")
    # band solver with row swaps
    rng = np.random.default_rng(4)
    n = 40
    lo, di, up, rhs = (rng.standard_normal(n) for _ in range(4))
    lo[0] = 0.0
    up[-1] = 0.0
    di *= 0.2
    A = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    out = np.zeros(n)
    L.oracle_band_solve(n, _p(lo), _p(di), _p(up), _p(rhs), _p(out))
    if np.max(np.abs(out - np.linalg.solve(A, rhs))) > 1e-9 * (1 + np.max(np.abs(out))):
        failed.append("band")
    # the natural sentinel is strict
    x, y = w.paper_curve(np.random.default_rng(9), 10)
    rc, _, ypp = spline(x, y, 0.99e30, 1e32, 4)
    if rc or ypp[0] == 0.0:
        failed.append("sentinel")
    return failed


def _source():
    with open(oracle.SRC) as f:
        return f.read()


def test_unmutated_oracle_passes_battery():
    assert _battery(_compile(_source(), "orig")) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    src = _source()
    assert src.count(old) == 1, "mutation site not found: %s" % name
    L = _compile(src.replace(old, new), name)
    assert _battery(L), "planted mistake %s passed every pin" % name
