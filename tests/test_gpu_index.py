"""Step a5 (bracketing) on the kernels the product path runs, bit for bit.

spline_solve_uniform_indexed and spline_plan_run_indexed run the same kernels
as spline_solve_uniform and spline_plan_run, chosen by the same rules, with
one more store per result: the interval each kernel decided for each query.
The intervals must equal the oracle's binary search exactly, on knots placed
exactly on uniform query positions and one ulp to either side (where a wrong
query rounding or tie-break moves a query to the neighbouring interval), at
densities that route to every single-curve kernel and with every batched
tuning; the values must equal the unindexed launch's bit for bit.  The
full-size configurations compare every query, chunk by chunk."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import api, _native, workloads as w

pytestmark = pytest.mark.gpu


def knots_on_queries(seed, n, m):
    """n strictly increasing knots on [0, n - 1] (mean width 1); as many
    interior knots as there are interior queries sit exactly on uniform query
    positions of m queries, every third of those one ulp below and every third
    one ulp above; the rest are random."""
    rng = np.random.default_rng(seed)
    length = float(n - 1)
    q = oracle.uniform_queries(0.0, length, m)
    on = min(n - 2, max(m - 2, 0))
    ks = np.sort(rng.choice(np.arange(1, m - 1), on, replace=False)) if on > 0 else np.zeros(0, np.int64)
    pts = q[ks]
    sel = np.arange(on) % 3
    pts = np.where(sel == 1, np.nextafter(pts, -np.inf), pts)
    pts = np.where(sel == 2, np.nextafter(pts, np.inf), pts)
    x = np.unique(np.concatenate([[0.0, length], pts]))
    while len(x) < n:
        extra = rng.uniform(0.0, length, n - len(x))
        x = np.unique(np.concatenate([x, extra]))
    if len(x) > n:  # drop random interior extras, keep the ends and the on-query knots
        keep = np.isin(x, np.concatenate([[0.0, length], pts]))
        drop = rng.choice(np.nonzero(~keep)[0], len(x) - n, replace=False)
        x = np.delete(x, drop)
    assert len(x) == n and np.all(np.diff(x) > 0)
    y = rng.standard_normal(n)
    return x, y


def solve_indexed(x, y, sd, ed, m):
    xd, yd = dev(x), dev(y)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    ypp = torch.full_like(xd, np.nan)
    idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    api.spline_solve_uniform_indexed(xd, yd, sd, ed, m, yq, idx, ypp, st)
    yq0 = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    ypp0 = torch.full_like(xd, np.nan)
    api.spline_solve_uniform(xd, yd, sd, ed, m, yq0, ypp0)
    assert int(host(st)[0]) == api.OK
    return host(yq), host(idx), host(ypp), host(yq0), host(ypp0)


# (n, m) -> the kernel spline_solve_uniform picks (256 compute units):
#   cooperative (>= 10 queries per interval, few blocks, or >= 1024 per
#   interval), wavefront per block (>= 10, more than 32 blocks per compute
#   unit), block kernel (< 10, shorter curves), streaming kernel (< 4 from
#   163,840 knots, < 10 from 2^20)
ROUTES = {
    "coop": [(13, 2048), (4001, 400000), (1001, 2000000), (65, 1 << 20)],
    "waves": [(300001, 3600001)],
    "blocks": [(3, 5), (20001, 100000), (5000, 3), (4097, 333), (70001, 70000)],
    "stream": [(200001, 400000), ((1 << 20) + 1, 8000000), (1 << 18, 7), (300001, 2)],
}


@pytest.mark.parametrize("route,n,m", [(r, n, m) for r, cases in ROUTES.items() for n, m in cases])
def test_single_curve_intervals_bit_exact(route, n, m):
    x, y = knots_on_queries(n + 7 * m, n, m)
    sd, ed = (1e32, 1e32) if (n + m) % 2 else (-1.0, 0.5)
    g_yq, g_idx, g_ypp, yq0, ypp0 = solve_indexed(x, y, sd, ed, m)
    np.testing.assert_array_equal(g_idx, oracle.bracket_uniform(x, m), "%s n=%d m=%d" % (route, n, m))
    np.testing.assert_array_equal(g_yq, yq0)
    np.testing.assert_array_equal(g_ypp, ypp0)
    o_yq, o_ypp = oracle.spline_uniform(x, y, sd, ed, m)
    assert_close(g_ypp, o_ypp, "ypp %s" % route)
    assert_close(g_yq, o_yq, "yq %s" % route)


def test_stream_wide_intervals_bit_exact():
    # the streaming kernel's whole-wavefront path (an interval with more than
    # 32 queries) next to the per-lane walk, with knots on query positions
    n, m = (1 << 18) + 3, 3 << 18
    x, y = knots_on_queries(5, n, m)
    widths = np.diff(x)
    for j in (9, 1000, 77777, n - 5):
        widths[j] *= 400.0
    x = np.concatenate([[0.0], np.cumsum(widths)])
    g_yq, g_idx, _, yq0, _ = solve_indexed(x, y, 0.0, 0.0, m)
    np.testing.assert_array_equal(g_idx, oracle.bracket_uniform(x, m))
    np.testing.assert_array_equal(g_yq, yq0)


def batch_on_queries(seed, sizes):
    xs, ys, koff, qoff = [], [], [0], [0]
    for i, (n, m) in enumerate(sizes):
        x, y = knots_on_queries(seed + i, n, m)
        xs.append(x)
        ys.append(y)
        koff.append(koff[-1] + n)
        qoff.append(qoff[-1] + m)
    count = len(sizes)
    sd = np.array([w.bc_for(i)[1] for i in range(count)])
    ed = np.array([w.bc_for(i)[2] for i in range(count)])
    return np.concatenate(xs), np.concatenate(ys), sd, ed, np.array(koff, np.int64), np.array(qoff, np.int64)


BATCH_SIZES = ([(3, 1), (3, 2), (4, 7), (13, 2048), (64, 64), (65, 30000), (128, 20480), (129, 5),
                (256, 100000), (257, 3000), (512, 9000), (513, 40000), (1300, 204800), (2048, 5000),
                (2047, 2), (700, 90)] +
               [(int(n), int(m)) for n, m in zip(*w.log_uniform_sizes(np.random.default_rng(2), 200, 0.1, 10))])

TUNINGS = [None, (256, 8192, 0, 1), (64, 2048, 16, 1), (256, 4096, 0, 2), (256, 8192, 0, 3), (256, 8192, 0, 4)]


@pytest.mark.parametrize("tuning", TUNINGS)
@pytest.mark.parametrize("precision", [api.FP64, api.FP32_REFINE])
def test_batched_intervals_bit_exact(tuning, precision):
    x, y, sd, ed, koff, qoff = batch_on_queries(100, BATCH_SIZES)
    t = _native.Tuning(*tuning) if tuning else None
    plan = api.spline_plan_create(koff, qoff, precision=precision, tuning=t)
    bufs = {"x": dev(x), "y": dev(y), "sd": dev(sd), "ed": dev(ed), "koff": dev(koff, torch.int64),
            "qoff": dev(qoff, torch.int64),
            "yq": torch.full((int(qoff[-1]),), np.nan, dtype=torch.float64, device="cuda"),
            "ypp": torch.full((int(koff[-1]),), np.nan, dtype=torch.float64, device="cuda")}
    idx = torch.full((int(qoff[-1]),), -1, dtype=torch.int32, device="cuda")
    api.spline_plan_run_indexed(plan, bufs, idx)
    g_idx, g_yq = host(idx), host(bufs["yq"])
    bufs0 = dict(bufs, yq=torch.full_like(bufs["yq"], np.nan), ypp=torch.full_like(bufs["ypp"], np.nan))
    api.spline_plan_run(plan, bufs0)
    np.testing.assert_array_equal(g_yq, host(bufs0["yq"]))
    for i in range(len(BATCH_SIZES)):
        xi = x[koff[i]:koff[i + 1]]
        mi = int(qoff[i + 1] - qoff[i])
        np.testing.assert_array_equal(g_idx[qoff[i]:qoff[i + 1]], oracle.bracket_uniform(xi, mi),
                                      "curve %d (n=%d, m=%d)" % (i, len(xi), mi))
    if precision == api.FP64:
        o_yq, o_ypp, _, _ = oracle.batch_uniform(koff, qoff, x, y, sd, ed)
        for i in range(0, len(BATCH_SIZES), 5):
            assert_close(g_yq[qoff[i]:qoff[i + 1]], o_yq[qoff[i]:qoff[i + 1]], "batched yq %d" % i)


def compare_every_query(x, y, o_ypp, m, g_yq, g_idx, what, chunk=1 << 24):
    """Every query of the curve against the oracle, chunk by chunk (values
    within the tolerance, scaled by the whole curve's max |y_q|; intervals
    equal)."""
    scale = None
    worst = 0.0
    errs = []
    for k0 in range(0, m, chunk):
        k1 = min(m, k0 + chunk)
        o_v, o_i = oracle.uniform_range(x, y, o_ypp, m, k0, k1)
        np.testing.assert_array_equal(g_idx[k0:k1], o_i, "%s intervals [%d, %d)" % (what, k0, k1))
        errs.append((k0, k1, np.abs(g_yq[k0:k1] - o_v), np.abs(o_v)))
        mx = float(np.max(np.abs(o_v)))
        scale = mx if scale is None else max(scale, mx)
    for k0, k1, err, ao in errs:
        bad = err > 1e-10 * (ao + scale)
        assert not bad.any(), "%s: %d of queries [%d, %d) off, worst %.3e" % (
            what, int(bad.sum()), k0, k1, float(np.max(err / (ao + scale))))
        worst = max(worst, float(np.max(err / (ao + scale))))
    return worst


@pytest.mark.parametrize("n,m", [(13000, 1 << 27), (1 << 22, 47 << 22), (1 << 24, 1 << 24), (1 << 26, 1 << 26),
                                 (1 << 28, 1 << 28)])
def test_full_size_every_query(n, m):
    # the out-of-cache single-curve point (m = 2^27, the cooperative kernel),
    # a dense long curve (the wavefront-per-block kernel) and the size sweep's
    # points past the last-level cache (m = n, the streaming kernel, up to
    # its largest, 2^28): every y'', every query value and every interval
    x, y = w.paper_curve(np.random.default_rng(n % 1000 + 7), n)
    xd, yd = dev(x), dev(y)
    ypp = torch.empty_like(xd)
    yq = torch.empty(m, dtype=torch.float64, device="cuda")
    idx = torch.empty(m, dtype=torch.int32, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    api.spline_solve_uniform_indexed(xd, yd, 1e32, 1e32, m, yq, idx, ypp, st)
    assert int(host(st)[0]) == api.OK
    g_idx = host(idx)
    del idx
    g_yq = host(yq)
    # the unindexed launch gives the same values
    api.spline_solve_uniform(xd, yd, 1e32, 1e32, m, yq, ypp)
    same = torch.equal(yq, torch.from_numpy(g_yq).cuda())
    del yq, xd, yd
    assert same
    g_ypp = host(ypp)
    del ypp
    o_ypp = oracle.second_derivatives(x, y, 1e32, 1e32)
    assert_close(g_ypp, o_ypp, "full-size ypp n=%d" % n)
    compare_every_query(x, y, o_ypp, m, g_yq, g_idx, "n=%d m=%d" % (n, m))


@pytest.mark.parametrize("kind", ["random", "sorted", "on_knots", "outside"])
def test_eval_points_long_curve(kind):
    # explicit points on a curve of 2^20 + 3 knots: sorted points reach the
    # kernel's staged-window path (a tile's points span a few hundred knots),
    # random ones its search over the whole knot array; values, first and
    # second derivatives, and intervals bit for bit
    n = (1 << 20) + 3
    x, y = w.paper_curve(np.random.default_rng(50), n)
    sd, ed = -1.0, 0.5
    rng = np.random.default_rng(51)
    if kind == "random":
        q = rng.uniform(x[0], x[-1], 1 << 22)
    elif kind == "sorted":
        q = np.sort(rng.uniform(x[0], x[-1], 1 << 22))
    elif kind == "on_knots":
        q = np.concatenate([x[::4], np.nextafter(x[1::4], np.inf), np.nextafter(x[2::4], -np.inf)])
        q = q[rng.permutation(len(q))]
    else:
        q = rng.uniform(x[0] - 10.0, x[-1] + 10.0, 1 << 20)
    m = len(q)
    xd, yd = dev(x), dev(y)
    ypp = torch.full_like(xd, np.nan)
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    api.spline_solve_uniform(xd, yd, sd, ed, 1, one, ypp)
    qd = dev(q)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    d1 = torch.full_like(yq, np.nan)
    d2 = torch.full_like(yq, np.nan)
    idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    api.spline_eval_points(xd, yd, ypp, qd, yq, d1, d2, idx)
    o_ypp = oracle.second_derivatives(x, y, sd, ed)
    assert_close(host(ypp), o_ypp, "points ypp")
    o_yq, o_idx = oracle.eval_points(x, y, o_ypp, q, with_index=True)
    o_d1, o_d2 = oracle.eval_points_derivs(x, y, o_ypp, q)
    np.testing.assert_array_equal(host(idx), o_idx, kind)
    assert_close(host(yq), o_yq, "yq points " + kind)
    assert_close(host(d1), o_d1, "d1 points " + kind, rtol=1e-9)
    assert_close(host(d2), o_d2, "d2 points " + kind, rtol=1e-9)
