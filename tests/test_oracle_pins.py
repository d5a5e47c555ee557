"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * the values the paper prints (Table tbl:test_compare_nat1; the error
    magnitudes of the "Quality Checks" tables),
  * an exact rational solve of the textbook spline conditions (tests/exact_spline.py),
  * closed forms (cubic reproduction, linear data, uniform knots),
  * SciPy's CubicSpline, a library routine for the same special cases,
  * invariants (interpolation, C1/C2 continuity, end slopes, residual),
  * brute force for the integer bracketing step,
  * a dense LAPACK solve for the band solver.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.interpolate as si

import oracle
from exact_spline import ExactSpline
from paper_2001_09253_amd import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BCS = [(1e32, 1e32), (0.0, 0.0), (-1.0, 1.0), (1e32, 0.5), (-2.0, np.inf)]


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _rand_curve(seed, n):
    return w.paper_curve(np.random.default_rng(seed), n)


# -- values the paper prints ------------------------------------------------------------

def test_table1_natural_second_derivatives():
    rows = _golden("table1_natural_ypp.txt")
    x = np.array([float(r[0]) for r in rows])
    y = np.array([float(r[1]) for r in rows])
    printed = np.array([float(r[2]) for r in rows])
    np.testing.assert_array_equal(x, w.HAND_KNOTS)
    np.testing.assert_array_equal(y, w.HAND_VALUES)
    ypp = oracle.second_derivatives(x, y, 1e32, 1e32)
    # printed to 6 decimals: half a unit in the last printed place
    assert np.max(np.abs(ypp - printed)) <= 5e-7 + 1e-12


@pytest.mark.parametrize("case", ["natural", "flat", "twist", "curve"])
def test_error_magnitudes_match_paper(case):
    row = next(r for r in _golden("error_magnitudes.txt") if r[0] == case)
    sd, ed = float(row[1]), float(row[2])
    max_delta, mse_nr, mse_our = float(row[3]), float(row[4]), float(row[5])
    ex = ExactSpline(w.HAND_KNOTS, w.HAND_VALUES, sd, ed)
    if case == "curve":
        yq, _ = oracle.spline_uniform(w.HAND_KNOTS, w.HAND_VALUES, sd, ed, 2048)
        q = oracle.uniform_queries(w.HAND_KNOTS[0], w.HAND_KNOTS[-1], 2048)
        truth = np.array([float(ex.value(Fraction(float(v)))) for v in q])
        err = yq - truth
    else:
        ypp = oracle.second_derivatives(w.HAND_KNOTS, w.HAND_VALUES, sd, ed)
        truth = np.array([float(v) for v in ex.second_derivatives()])
        err = ypp - truth
        # the paper's largest FP64 delta is a few 1e-13; allow one order more
        assert np.max(np.abs(err)) <= 10 * max_delta
    mse = float(np.mean(err ** 2))
    # "chaotic" rounding: only the order of magnitude is pinned
    assert mse <= 100 * max(mse_nr, mse_our)


# -- exact rational brute force ------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_exact_rational_spline(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 9))
    x, y = _rand_curve(seed, n)
    sd, ed = BCS[seed % len(BCS)]
    ex = ExactSpline(x, y, sd, ed)
    truth = np.array([float(v) for v in ex.second_derivatives()])
    ypp = oracle.second_derivatives(x, y, sd, ed)
    scale = np.max(np.abs(truth)) + 1e-300
    assert np.max(np.abs(ypp - truth)) <= 1e-13 * scale
    m = int(rng.integers(2, 60))
    yq, _ = oracle.spline_uniform(x, y, sd, ed, m)
    q = oracle.uniform_queries(x[0], x[-1], m)
    tv = np.array([float(ex.value(Fraction(float(v)))) for v in q])
    assert np.max(np.abs(yq - tv)) <= 1e-13 * (np.max(np.abs(tv)) + scale * (x[-1] - x[0]) ** 2)


@pytest.mark.parametrize("n", [24, 40])
def test_exact_rational_spline_longer(n):
    # two longer curves (the rational solve grows as n^3: n = 40 takes seconds)
    x, y = _rand_curve(500 + n, n)
    for sd, ed in (BCS[0], BCS[2]):
        ex = ExactSpline(x, y, sd, ed)
        truth = np.array([float(v) for v in ex.second_derivatives()])
        ypp = oracle.second_derivatives(x, y, sd, ed)
        assert np.max(np.abs(ypp - truth)) <= 1e-13 * (np.max(np.abs(truth)) + 1e-300)


def test_exact_rational_wild_spacing():
    # intervals from 1e-9 to 1e3 in one curve
    x = np.array([0.0, 1e-9, 1.0, 1.0 + 1e-6, 1000.0, 1000.5, 2000.0])
    y = np.array([0.3, -0.7, 0.1, 0.9, 0.2, 0.25, -0.4])
    for sd, ed in BCS:
        ex = ExactSpline(x, y, sd, ed)
        truth = np.array([float(v) for v in ex.second_derivatives()])
        ypp = oracle.second_derivatives(x, y, sd, ed)
        assert np.max(np.abs(ypp - truth)) <= 1e-10 * np.max(np.abs(truth))


# -- closed forms ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_clamped_cubic_is_reproduced(seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-2, 2, size=4)
    p = np.polynomial.Polynomial(c)
    x, _ = _rand_curve(seed + 50, 40)
    y = p(x)
    dp, ddp = p.deriv(1), p.deriv(2)
    ypp = oracle.second_derivatives(x, y, dp(x[0]), dp(x[-1]))
    scale = np.max(np.abs(ddp(x)))
    assert np.max(np.abs(ypp - ddp(x))) <= 1e-9 * scale
    yq, _ = oracle.spline_uniform(x, y, dp(x[0]), dp(x[-1]), 777)
    q = oracle.uniform_queries(x[0], x[-1], 777)
    assert np.max(np.abs(yq - p(q))) <= 1e-9 * np.max(np.abs(p(q)))


def test_natural_linear_data_is_linear():
    x, _ = _rand_curve(7, 64)
    y = 3.0 * x - 2.0
    ypp = oracle.second_derivatives(x, y, 1e32, 1e32)
    assert np.max(np.abs(ypp)) <= 1e-10
    yq, _ = oracle.spline_uniform(x, y, 1e32, 1e32, 1000)
    q = oracle.uniform_queries(x[0], x[-1], 1000)
    assert np.max(np.abs(yq - (3.0 * q - 2.0))) <= 1e-11 * np.max(np.abs(y))


def test_uniform_knots_textbook_system():
    # equal spacing h: interior rows become y''_{j-1} + 4 y''_j + y''_{j+1} = 6 (y_{j+1} - 2 y_j + y_{j-1}) / h^2
    h = 0.25
    x = np.arange(20) * h
    y = np.sin(3 * x) + 0.1 * np.random.default_rng(3).random(20)
    ypp = oracle.second_derivatives(x, y, 1e32, 1e32)
    lhs = ypp[:-2] + 4 * ypp[1:-1] + ypp[2:]
    rhs = 6 * (y[2:] - 2 * y[1:-1] + y[:-2]) / h ** 2
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * np.max(np.abs(rhs))
    assert ypp[0] == 0.0 and ypp[-1] == 0.0


# -- a library routine for the same special cases -------------------------------------------

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("bc", range(len(BCS)))
def test_scipy_cubicspline(seed, bc):
    sd, ed = BCS[bc]
    n = [3, 4, 13, 100, 1000, 5][seed]
    x, y = _rand_curve(seed, n)
    bct = (
        (2, 0.0) if sd > 0.99e30 else (1, sd),
        (2, 0.0) if ed > 0.99e30 else (1, ed),
    )
    cs = si.CubicSpline(x, y, bc_type=bct)
    ypp = oracle.second_derivatives(x, y, sd, ed)
    ref = cs(x, 2)
    assert np.max(np.abs(ypp - ref)) <= 1e-12 * (np.max(np.abs(ref)) + 1.0)
    m = 3 * n + 7
    yq, _ = oracle.spline_uniform(x, y, sd, ed, m)
    q = oracle.uniform_queries(x[0], x[-1], m)
    assert np.max(np.abs(yq - cs(q))) <= 1e-12 * (np.max(np.abs(cs(q))) + np.max(np.abs(ref)))
    d1, d2 = oracle.eval_points_derivs(x, y, ypp, q)
    assert np.max(np.abs(d1 - cs(q, 1))) <= 1e-11 * (np.max(np.abs(cs(q, 1))) + np.max(np.abs(ref)))
    assert np.max(np.abs(d2 - cs(q, 2))) <= 1e-11 * (np.max(np.abs(ref)) + 1.0)


# -- invariants -----------------------------------------------------------------------------

@pytest.mark.parametrize("bc", range(len(BCS)))
def test_spline_invariants(bc):
    sd, ed = BCS[bc]
    x, y = _rand_curve(11 + bc, 200)
    ypp = oracle.second_derivatives(x, y, sd, ed)
    scale = np.max(np.abs(ypp)) + 1.0
    # interpolation at every knot (from both neighbouring intervals)
    for j in range(len(x)):
        for i in (j - 1, j):
            if 0 <= i <= len(x) - 2:
                v, _, d2 = oracle.eval_on_interval(x, y, ypp, i, x[j])
                assert abs(v - y[j]) <= 1e-13 * (1 + abs(y[j])) + 1e-15 * scale
                assert abs(d2 - ypp[j]) <= 1e-12 * scale
    # first-derivative continuity at interior knots: the row equation itself
    for j in range(1, len(x) - 1):
        _, left, _ = oracle.eval_on_interval(x, y, ypp, j - 1, x[j])
        _, right, _ = oracle.eval_on_interval(x, y, ypp, j, x[j])
        assert abs(left - right) <= 1e-11 * scale
    # the ends behave per end
    _, d1s, d2s = oracle.eval_on_interval(x, y, ypp, 0, x[0])
    _, d1e, d2e = oracle.eval_on_interval(x, y, ypp, len(x) - 2, x[-1])
    if sd > 0.99e30:
        assert d2s == 0.0
    else:
        assert abs(d1s - sd) <= 1e-11 * scale
    if ed > 0.99e30:
        assert d2e == 0.0
    else:
        assert abs(d1e - ed) <= 1e-11 * scale
    # residual of the assembled system
    lo, di, up, rhs = oracle.rows(x, y, sd, ed)
    r = di * ypp - rhs
    r[1:] += lo[1:] * ypp[:-1]
    r[:-1] += up[:-1] * ypp[1:]
    tn = np.max(np.abs(lo) + np.abs(di) + np.abs(up))
    assert np.max(np.abs(r)) <= 1e-14 * (tn * np.max(np.abs(ypp)) + np.max(np.abs(rhs)))


def test_simple_boundary_equals_flat_clamp():
    # The paper's first routine (x_0 = x_1 trick) is the clamped routine with
    # zero end slopes; in terms of rows: b_1 = 2 c_1, d_1 = 6 slope.
    x, y = _rand_curve(5, 30)
    lo, di, up, rhs = oracle.rows(x, y, 0.0, 0.0)
    h0, hn = x[1] - x[0], x[-1] - x[-2]
    assert di[0] == 2 * h0 and up[0] == h0 and rhs[0] == 6 * ((y[1] - y[0]) / h0)
    assert lo[-1] == hn and di[-1] == 2 * hn and rhs[-1] == -6 * ((y[-1] - y[-2]) / hn)


# -- band solver against a dense solve (with pivoting exercised) -----------------------------

@pytest.mark.parametrize("seed", range(6))
def test_band_solve_dense(seed):
    rng = np.random.default_rng(seed)
    n = [1, 2, 3, 7, 50, 300][seed]
    lo, di, up, rhs = (rng.standard_normal(n) for _ in range(4))
    lo[0] = 0.0
    up[-1] = 0.0
    di *= 0.2        # not diagonally dominant: row swaps happen
    A = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    ref = np.linalg.solve(A, rhs)
    out = oracle.band_solve(lo, di, up, rhs)
    assert np.max(np.abs(out - ref)) <= 1e-9 * (1 + np.max(np.abs(ref)))


# -- bracketing and queries: integer work, bit-exact -----------------------------------------

def _scan_bracket(x, qs):
    """The paper's bracketing loop: advance while the next knot is below q."""
    out = []
    i = 0
    for q in qs:
        while i + 1 < len(x) - 1 and x[i + 1] < q:
            i += 1
        out.append(i)
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_bracket_matches_scan(seed):
    n = [3, 4, 13, 200, 1000][seed]
    x, _ = _rand_curve(seed, n)
    m = [2, 5, 2048, 1999, 1000][seed]
    idx = oracle.bracket_uniform(x, m)
    q = oracle.uniform_queries(x[0], x[-1], m)
    np.testing.assert_array_equal(idx, _scan_bracket(x, q))
    # queries exactly on knots and one ulp either side
    qs = np.sort(np.concatenate([x, np.nextafter(x, -np.inf), np.nextafter(x, np.inf)]))
    np.testing.assert_array_equal([oracle.bracket(x, v) for v in qs], _scan_bracket(x, qs))
    for v in qs:
        i = oracle.bracket(x, v)
        cnt = int(np.sum(x < v))
        assert i == min(max(cnt - 1, 0), n - 2)


# (x0, x_last, m): the worked size, m = 1 and 2, wide and narrow ranges, a
# negative range, and C2's 2,048,000 queries
QUERY_CASES = [(0.0, 2.5, 2048), (-3.0, 7.25, 1), (1.0, 2.0, 2), (0.1, 1e6, 100003), (0.0, 13.0, 2048),
               (-1e-3, 5e5, 2048000), (3.7, 3.7000001, 999), (-7.5, -0.25, 65537), (0.0, 1.0, 11)]


@pytest.mark.parametrize("x0,x1,m", QUERY_CASES)
def test_uniform_queries_are_linspace_bit_for_bit(x0, x1, m):
    # The paper samples its interpolated curve with np.linspace(min, max,
    # 2048) ("Quality Checks"); the oracle's positions must be those bits
    # exactly (one multiply, then one add, never fused; the last query is
    # x_last itself), since the bracketing of on-knot queries depends on them.
    q = oracle.uniform_queries(x0, x1, m)
    np.testing.assert_array_equal(q, np.linspace(x0, x1, m))
    assert q[0] == x0
    if m > 1:
        assert q[-1] == x1
        assert np.all(np.diff(q) >= 0)
    for k in {0, 1, m // 2, m - 2, m - 1}:
        if 0 <= k < m:
            assert oracle.uniform_query(x0, x1, m, k) == q[k]


def test_uniform_queries_of_the_worked_example():
    # the worked example's own call: 2048 points between the first and last
    # of the 13 hand knots
    q = oracle.uniform_queries(w.HAND_KNOTS[0], w.HAND_KNOTS[-1], 2048)
    np.testing.assert_array_equal(q, np.linspace(min(w.HAND_KNOTS), max(w.HAND_KNOTS), 2048))


def test_validation_codes():
    assert oracle.validate(np.array([0.0, 1.0])) == oracle.E_SIZE
    assert oracle.validate(np.array([0.0, 1.0, 1.0])) == oracle.E_ORDER
    assert oracle.validate(np.array([0.0, 2.0, 1.0])) == oracle.E_ORDER
    assert oracle.validate(np.array([0.0, np.nan, 1.0])) == oracle.E_ORDER
    assert oracle.validate(np.array([0.0, 1.0, 2.0])) == oracle.OK
    with pytest.raises(oracle.OracleError):
        oracle.second_derivatives([0.0, 1.0], [1.0, 2.0], 0.0, 0.0)


def test_natural_sentinel_is_strict_and_per_end():
    x, y = _rand_curve(9, 10)
    a = oracle.second_derivatives(x, y, 0.99e30, 1e32)
    b = oracle.second_derivatives(x, y, 1e31, 1e32)
    assert b[0] == 0.0 and b[-1] == 0.0
    assert a[0] != 0.0          # 0.99e30 itself is a (huge) clamped slope
    c = oracle.second_derivatives(x, y, np.inf, -1.0)
    assert c[0] == 0.0 and c[-1] != 0.0
    d = oracle.second_derivatives(x, y, np.nan, 1e32)
    assert np.all(np.isnan(d[:-1]))
