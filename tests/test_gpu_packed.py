"""Explicit points on a packed curve (spline_pack_knots, then
spline_eval_points_packed): the same kernel as spline_eval_points reading x,
y and y'' interleaved, so every interval must equal spline_eval_points' bit
for bit and every value and derivative to rounding (the two instantiations'
compiled code may contract a multiply and an add differently), and the
oracle's within the tolerance, on the long curve (the fence table and the
search in global memory) and on a short one, for random, sorted, on-knot,
outside and NaN points."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import api, workloads as w

pytestmark = pytest.mark.gpu


def points(x, kind, rng, m):
    if kind == "random":
        return rng.uniform(x[0], x[-1], m)
    if kind == "sorted":
        return np.sort(rng.uniform(x[0], x[-1], m))
    if kind == "on_knots":
        pick = x[rng.integers(0, len(x), m)]
        sel = rng.integers(0, 3, m)
        return np.where(sel == 1, np.nextafter(pick, -np.inf), np.where(sel == 2, np.nextafter(pick, np.inf), pick))
    if kind == "outside":
        return rng.uniform(x[0] - 10.0, x[-1] + 10.0, m)
    q = rng.uniform(x[0], x[-1], m)
    q[np.arange(7, m, 3 * 4096)] = np.nan
    return q


def run(fn, m):
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    d1 = torch.full_like(yq, np.nan)
    d2 = torch.full_like(yq, np.nan)
    idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    fn(yq, d1, d2, idx)
    return [host(t) for t in (yq, d1, d2, idx)]


@pytest.mark.parametrize("n", [777, (1 << 20) + 3])
@pytest.mark.parametrize("kind", ["random", "sorted", "on_knots", "outside", "nan"])
def test_packed_equals_unpacked(n, kind):
    rng = np.random.default_rng(n % 1000 + len(kind))
    x, y = w.paper_curve(rng, n)
    sd, ed = 1e32, -0.5
    xd, yd = dev(x), dev(y)
    ypp = torch.full_like(xd, np.nan)
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    api.spline_solve_uniform(xd, yd, sd, ed, 1, one, ypp)
    packed = torch.full((3 * n,), np.nan, dtype=torch.float64, device="cuda")
    api.spline_pack_knots(xd, yd, ypp, packed)
    np.testing.assert_array_equal(host(packed).reshape(n, 3), np.stack([x, y, host(ypp)], axis=1))
    q = points(x, kind, rng, 1 << 20 if n > 1000 else 100000)
    qd = dev(q)
    m = len(q)
    a = run(lambda yq, d1, d2, idx: api.spline_eval_points(xd, yd, ypp, qd, yq, d1, d2, idx), m)
    b = run(lambda yq, d1, d2, idx: api.spline_eval_points_packed(packed, qd, yq, d1, d2, idx), m)
    np.testing.assert_array_equal(a[3], b[3], "intervals %s n=%d" % (kind, n))
    fin = np.isfinite(q)
    for g, h, what in zip(a[:3], b[:3], ("yq", "d1", "d2")):
        assert np.all(np.isnan(g[~fin])) and np.all(np.isnan(h[~fin])), (n, kind, what)
        assert_close(h[fin], g[fin], "packed against unpacked %s %s n=%d" % (what, kind, n), rtol=1e-14)
    # and the oracle, on finite points
    o_ypp = oracle.second_derivatives(x, y, sd, ed)
    o_yq, o_idx = oracle.eval_points(x, y, o_ypp, q, with_index=True)
    np.testing.assert_array_equal(b[3], o_idx)
    assert_close(b[0][fin], o_yq[fin], "packed yq %s n=%d" % (kind, n))
