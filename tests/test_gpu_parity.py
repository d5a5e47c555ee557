"""Parity of the HIP path (through the C ABI) with the FP64 oracle, one curve
at a time: build (a1-a4), uniform evaluate (a5-a6), bracketing (bit-exact),
the noop loop, explicit queries and their derivatives."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import RTOL, assert_close, dev, host
from paper_2001_09253_amd import api, workloads as w

pytestmark = pytest.mark.gpu

BCS = [("natural", 1e32, 1e32), ("flat", 0.0, 0.0), ("twist", -1.0, 1.0), ("mixed", 1e32, 0.5),
       ("mixed2", -2.0, np.inf)]
SIZES = [3, 4, 5, 13, 63, 64, 65, 100, 256, 257, 1000, 1024, 1025, 4096, 4097, 8192, 8193, 13000, 16384]


def gpu_build(x, y, sd, ed):
    xd, yd = dev(x), dev(y)
    ypp = torch.full_like(xd, np.nan)
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    api.spline_build(xd, yd, sd, ed, ypp, st)
    return host(ypp), int(host(st)[0]), (xd, yd, ypp)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bc", range(len(BCS)))
def test_build_matches_oracle(n, bc):
    name, sd, ed = BCS[bc]
    x, y = w.paper_curve(np.random.default_rng(n * 7 + bc), n)
    g, st, _ = gpu_build(x, y, sd, ed)
    assert st == api.OK
    o = oracle.second_derivatives(x, y, sd, ed)
    assert_close(g, o, "ypp n=%d %s" % (n, name))
    if sd > 0.99e30:
        assert g[0] == 0.0
    if ed > 0.99e30:
        assert g[-1] == 0.0


def test_build_hand_curve_table1():
    g, st, _ = gpu_build(w.HAND_KNOTS, w.HAND_VALUES, 1e32, 1e32)
    o = oracle.second_derivatives(w.HAND_KNOTS, w.HAND_VALUES, 1e32, 1e32)
    assert_close(g, o, "hand curve")


@pytest.mark.parametrize("scale", [1e-12, 1e-6, 1.0, 1e6])
def test_build_extreme_spacing(scale):
    rng = np.random.default_rng(3)
    inc = rng.random(3000) * scale
    inc[::97] *= 1e-6          # clusters of nearly coincident knots
    inc[inc == 0] = scale
    x = np.cumsum(inc)
    y = rng.standard_normal(3000)
    for _, sd, ed in BCS:
        g, st, _ = gpu_build(x, y, sd, ed)
        o = oracle.second_derivatives(x, y, sd, ed)
        assert_close(g, o, "spacing %g" % scale)


def test_build_rejects_unordered_knots():
    x, y = w.paper_curve(np.random.default_rng(1), 500)
    x1 = x.copy(); x1[200] = x1[199]              # repeated knot
    x2 = x.copy(); x2[10], x2[11] = x2[11], x2[10]  # swapped
    x3 = x.copy(); x3[499] = np.nan               # NaN
    for xb in (x1, x2, x3):
        g, st, _ = gpu_build(xb, y, 1e32, 1e32)
        assert st == api.E_ORDER
        assert np.all(np.isnan(g))


def test_build_size_limits():
    x = torch.zeros(api.MAX_N_BLOCK + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(api.SolveError) as e:
        api.spline_build(x, x, 0.0, 0.0, x)
    assert e.value.code == api.E_SIZE
    with pytest.raises(api.SolveError) as e:
        api.spline_build(x[:2], x[:2], 0.0, 0.0, x[:2])
    assert e.value.code == api.E_SIZE


def test_natural_sentinel_is_strict():
    x, y = w.paper_curve(np.random.default_rng(2), 50)
    g, _, _ = gpu_build(x, y, 0.99e30, 1e31)
    o = oracle.second_derivatives(x, y, 0.99e30, 1e31)
    assert g[0] != 0.0 and g[-1] == 0.0
    assert_close(g, o, "sentinel")


EVAL_CASES = [(13, 2048), (13, 1), (13, 2), (3, 5), (4, 4), (100, 1025), (1000, 1000), (5, 100003),
              (257, 4096 + 17), (4097, 3000), (13, 1024), (13, 1023), (13, 1025), (2000, 100)]


@pytest.mark.parametrize("n,m", EVAL_CASES)
@pytest.mark.parametrize("bc", [0, 2])
def test_eval_uniform_matches_oracle(n, m, bc):
    name, sd, ed = BCS[bc]
    x, y = w.paper_curve(np.random.default_rng(n + m), n)
    _, _, (xd, yd, ypp) = gpu_build(x, y, sd, ed)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    api.spline_eval_uniform(xd, yd, ypp, m, yq)
    o_yq, _ = oracle.spline_uniform(x, y, sd, ed, m)
    assert_close(host(yq), o_yq, "yq n=%d m=%d %s" % (n, m, name))


@pytest.mark.parametrize("n,m", EVAL_CASES + [(13000, 2048000), (16384, 7)])
def test_bracket_bit_exact(n, m):
    x, _ = w.paper_curve(np.random.default_rng(5 * n + m), n)
    idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    api.spline_bracket_uniform(dev(x), m, idx)
    np.testing.assert_array_equal(host(idx), oracle.bracket_uniform(x, m))


def test_bracket_queries_on_knots():
    # Place the knots exactly on uniform query positions (computed by the
    # oracle), and one ulp to either side: the interval choice then depends on
    # the exact query arithmetic and the strict comparison.
    m = 4001
    q = oracle.uniform_queries(0.0, 10.0, m)
    picks = np.sort(np.random.default_rng(9).choice(np.arange(1, m - 1), 600, replace=False))
    inner = q[picks]
    inner = np.where(np.arange(len(inner)) % 3 == 1, np.nextafter(inner, -np.inf), inner)
    inner = np.where(np.arange(len(inner)) % 3 == 2, np.nextafter(inner, np.inf), inner)
    x = np.unique(np.concatenate([[0.0], inner, [10.0]]))
    for mm in (m, 2 * m - 1):
        idx = torch.full((mm,), -1, dtype=torch.int32, device="cuda")
        api.spline_bracket_uniform(dev(x), mm, idx)
        np.testing.assert_array_equal(host(idx), oracle.bracket_uniform(x, mm))


def test_bracket_clustered_knots_wide_window():
    # Far more knots than queries: the tile's window exceeds the LDS and the
    # global-memory search path runs.
    x, _ = w.paper_curve(np.random.default_rng(4), 16000)
    for m in (3, 10, 999, 1025):
        idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
        api.spline_bracket_uniform(dev(x), m, idx)
        np.testing.assert_array_equal(host(idx), oracle.bracket_uniform(x, m))


def test_noop_reports_the_brackets():
    x, _ = w.paper_curve(np.random.default_rng(8), 1000)
    m = 50000
    out = torch.full((m,), -1.0, dtype=torch.float64, device="cuda")
    api.spline_noop_uniform(dev(x), m, out)
    np.testing.assert_array_equal(host(out), oracle.bracket_uniform(x, m).astype(np.float64))


def test_full_size_plain_config():
    inst = w.config_large(seed=0)
    _, _, (xd, yd, ypp) = gpu_build(inst.x, inst.y, inst.start_deriv, inst.end_deriv)
    yq = torch.full((inst.m,), np.nan, dtype=torch.float64, device="cuda")
    api.spline_eval_uniform(xd, yd, ypp, inst.m, yq)
    o_yq, o_ypp = oracle.spline_uniform(inst.x, inst.y, inst.start_deriv, inst.end_deriv, inst.m)
    assert_close(host(ypp), o_ypp, "ypp full size")
    assert_close(host(yq), o_yq, "yq full size")


def test_deterministic_repeat():
    inst = w.config_large(seed=1, bc=2)
    outs = []
    for _ in range(3):
        _, _, (xd, yd, ypp) = gpu_build(inst.x, inst.y, inst.start_deriv, inst.end_deriv)
        yq = torch.empty(inst.m, dtype=torch.float64, device="cuda")
        api.spline_eval_uniform(xd, yd, ypp, inst.m, yq)
        outs.append((host(ypp), host(yq)))
    for ypp_k, yq_k in outs[1:]:
        np.testing.assert_array_equal(ypp_k, outs[0][0])
        np.testing.assert_array_equal(yq_k, outs[0][1])


@pytest.mark.parametrize("kind", ["random", "sorted", "outside", "on_knots", "nan", "nan_sorted"])
def test_eval_points_matches_oracle(kind):
    n = 777
    x, y = w.paper_curve(np.random.default_rng(11), n)
    sd, ed = -1.0, 1.0
    _, _, (xd, yd, ypp) = gpu_build(x, y, sd, ed)
    rng = np.random.default_rng(12)
    if kind == "random":
        q = rng.uniform(x[0], x[-1], 100003)
    elif kind == "sorted":
        q = np.sort(rng.uniform(x[0], x[-1], 70001))
    elif kind == "outside":
        q = rng.uniform(x[0] - 5, x[-1] + 5, 5000)
    elif kind == "on_knots":
        q = np.concatenate([x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf)])
    elif kind == "nan":
        q = rng.uniform(x[0], x[-1], 3000)
        q[17] = np.nan
    else:
        # sorted points (tiles of 4096 whose knots fit the staged window)
        # with a NaN in every third tile: those tiles search everything,
        # their neighbours stay staged
        q = np.sort(rng.uniform(x[0], x[-1], 60000))
        q[np.arange(5, len(q), 3 * 4096)] = np.nan
    m = len(q)
    qd = dev(q)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    d1 = torch.full_like(yq, np.nan)
    d2 = torch.full_like(yq, np.nan)
    idx = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    api.spline_eval_points(xd, yd, ypp, qd, yq, d1, d2, idx)
    o_ypp = oracle.second_derivatives(x, y, sd, ed)
    o_yq, o_idx = oracle.eval_points(x, y, o_ypp, q, with_index=True)
    o_d1, o_d2 = oracle.eval_points_derivs(x, y, o_ypp, q)
    ok = ~np.isnan(q)
    np.testing.assert_array_equal(host(idx)[ok], o_idx[ok])
    assert_close(host(yq)[ok], o_yq[ok], "yq points " + kind)
    assert_close(host(d1)[ok], o_d1[ok], "d1 points " + kind, rtol=1e-9)
    assert_close(host(d2)[ok], o_d2[ok], "d2 points " + kind, rtol=1e-9)
    if not ok.all():
        assert np.all(np.isnan(host(yq)[~ok]))


SOLVE_CASES = [(3, 5), (13, 2048), (100, 7), (513, 100000), (1024, 1), (1025, 4096), (4097, 333),
               (13000, 2048000), (20000, 20000), (65536, 1 << 20), (300000, 1000), (250, 3000000),
               (300001, 19200000), (1 << 20, 1 << 16), (70001, 3), (100000, 800000)]


@pytest.mark.parametrize("n,m", SOLVE_CASES)
@pytest.mark.parametrize("bc", [0, 1, 2, 3])
def test_solve_uniform_matches_oracle(n, m, bc):
    name, sd, ed = BCS[bc]
    x, y = w.paper_curve(np.random.default_rng(3 * n + bc), n)
    xd, yd = dev(x), dev(y)
    ypp = torch.full_like(xd, np.nan)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    api.spline_solve_uniform(xd, yd, sd, ed, m, yq, ypp, st)
    o_yq, o_ypp = oracle.spline_uniform(x, y, sd, ed, m)
    assert int(host(st)[0]) == api.OK
    assert_close(host(ypp), o_ypp, "solve ypp n=%d %s" % (n, name))
    assert_close(host(yq), o_yq, "solve yq n=%d m=%d %s" % (n, m, name))


def test_solve_uniform_halo_worst_case_decay():
    # Widths shrinking by 1e-3 per knot make the forward error factor
    # a/(b - a c') approach its 2/3 bound; the halo must still be enough.
    n = 2000
    x, y = w.alternating_curve(np.random.default_rng(5), n, scale=1e3)
    for m in (n * 64, 3000):
        xd, yd = dev(x), dev(y)
        ypp = torch.empty_like(xd)
        yq = torch.empty(m, dtype=torch.float64, device="cuda")
        api.spline_solve_uniform(xd, yd, -1.0, 1.0, m, yq, ypp)
        o_yq, o_ypp = oracle.spline_uniform(x, y, -1.0, 1.0, m)
        assert_close(host(ypp), o_ypp, "decay ypp")
        assert_close(host(yq), o_yq, "decay yq")


@pytest.mark.parametrize("kind", ["sawtooth_down", "sawtooth_up", "loguniform", "clustered"])
@pytest.mark.parametrize("bc", [0, 3])
def test_solve_uniform_adaptive_halo_adversarial_spacing(kind, bc):
    # Dense queries take the kernel that sizes each block's halo from the
    # knots; these spacings keep the per-row decay factors near their bounds
    # in long runs.
    name, sd, ed = BCS[bc]
    n = 4000
    x, y = w.spacing_curve(np.random.default_rng(31 + bc), n, kind)
    for m in (n * 60, n * 400):
        xd, yd = dev(x), dev(y)
        ypp = torch.full_like(xd, np.nan)
        yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
        st = torch.zeros((1,), dtype=torch.int32, device="cuda")
        api.spline_solve_uniform(xd, yd, sd, ed, m, yq, ypp, st)
        o_yq, o_ypp = oracle.spline_uniform(x, y, sd, ed, m)
        assert int(host(st)[0]) == api.OK
        assert_close(host(ypp), o_ypp, "%s ypp m=%d %s" % (kind, m, name))
        assert_close(host(yq), o_yq, "%s yq m=%d %s" % (kind, m, name))


@pytest.mark.parametrize("kind", ["alternating", "sawtooth_down", "loguniform", "clustered"])
def test_solve_uniform_sparse_long_curves(kind):
    # long curves with far fewer queries than intervals take the block kernel
    # (256 intervals per block, per-query search); the alternating widths
    # force its uniform fallback halo (the widest span it holds)
    n, m = 70000, 3000
    rng = np.random.default_rng(41)
    if kind == "alternating":
        x, y = w.alternating_curve(rng, n, scale=10.0)
    else:
        x, y = w.spacing_curve(rng, n, kind)
    for sd, ed in ((1e32, 1e32), (-1.0, 2.0)):
        xd, yd = dev(x), dev(y)
        ypp = torch.full_like(xd, np.nan)
        yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
        st = torch.zeros((1,), dtype=torch.int32, device="cuda")
        api.spline_solve_uniform(xd, yd, sd, ed, m, yq, ypp, st)
        o_yq, o_ypp = oracle.spline_uniform(x, y, sd, ed, m)
        assert int(host(st)[0]) == api.OK
        assert_close(host(ypp), o_ypp, "%s sparse ypp" % kind)
        assert_close(host(yq), o_yq, "%s sparse yq" % kind)


def test_solve_uniform_sparse_bad_knots():
    x, y = w.paper_curve(np.random.default_rng(43), 100000)
    x[77777] = x[77776]
    xd, yd = dev(x), dev(y)
    yq = torch.empty(1000, dtype=torch.float64, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    api.spline_solve_uniform(xd, yd, 0.0, 0.0, 1000, yq, None, st)
    assert int(host(st)[0]) == api.E_ORDER


def test_solve_uniform_bad_knots_and_reuse():
    x, y = w.paper_curve(np.random.default_rng(21), 9000)
    xb = x.copy()
    xb[7000] = xb[6999]
    m = 300000
    o_yq, o_ypp = oracle.spline_uniform(x, y, -1.0, 1.0, m)
    for rep in range(3):
        for xx, good in ((x, True), (xb, False)):
            xd, yd = dev(xx), dev(y)
            ypp = torch.full_like(xd, 7.0)
            yq = torch.full((m,), 7.0, dtype=torch.float64, device="cuda")
            st = torch.zeros((1,), dtype=torch.int32, device="cuda")
            api.spline_solve_uniform(xd, yd, -1.0, 1.0, m, yq, ypp, st)
            if good:
                assert int(host(st)[0]) == api.OK
                assert_close(host(ypp), o_ypp, "reuse ypp")
                assert_close(host(yq), o_yq, "reuse yq")
            else:
                assert int(host(st)[0]) == api.E_ORDER


def test_solve_uniform_equals_two_launch_path():
    inst = w.config_large(seed=2, bc=1)
    xd, yd = dev(inst.x), dev(inst.y)
    ypp1 = torch.empty_like(xd)
    yq1 = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    api.spline_solve_uniform(xd, yd, inst.start_deriv, inst.end_deriv, inst.m, yq1, ypp1)
    ypp2 = torch.empty_like(xd)
    yq2 = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    api.spline_build(xd, yd, inst.start_deriv, inst.end_deriv, ypp2)
    api.spline_eval_uniform(xd, yd, ypp2, inst.m, yq2)
    assert_close(host(ypp1), host(ypp2), "one launch vs two", rtol=1e-12)
    assert_close(host(yq1), host(yq2), "one launch vs two", rtol=1e-12)


def test_solve_uniform_deterministic():
    inst = w.config_large(seed=3, bc=2)
    xd, yd = dev(inst.x), dev(inst.y)
    outs = []
    for _ in range(3):
        ypp = torch.empty_like(xd)
        yq = torch.empty(inst.m, dtype=torch.float64, device="cuda")
        api.spline_solve_uniform(xd, yd, inst.start_deriv, inst.end_deriv, inst.m, yq, ypp)
        outs.append((host(ypp), host(yq)))
    for ypp_k, yq_k in outs[1:]:
        np.testing.assert_array_equal(ypp_k, outs[0][0])
        np.testing.assert_array_equal(yq_k, outs[0][1])
