"""Parity of the batched form (the single-launch wave-item kernel over many
curves, hipGraph capture/replay, the autotuner) with the FP64 oracle, through
the C ABI."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import api, workloads as w

pytestmark = pytest.mark.gpu

# (block, queries_per_tile, grid_per_cu, fused)
TUNINGS = [(64, 64, 0, 1), (64, 1024, 2, 1), (128, 2048, 0, 1), (256, 4096, 0, 1), (256, 16384, 3, 1),
           (64, 64, 0, 2), (128, 1024, 2, 2), (256, 4096, 0, 2), (256, 16384, 5, 2),
           (256, 64, 0, 3), (256, 2048, 0, 3), (256, 16384, 0, 3),
           (256, 64, 0, 4), (256, 2048, 0, 4), (256, 8192, 0, 4), (256, 16384, 0, 4)]
# The two-launch form (a build kernel, then an evaluate kernel reading y''
# back) faulted the GPU in its build kernel with a memory aperture violation
# and no cause was found by reading it; it was taken out of the library, and
# its cases stay here, skipped, until it comes back with a found cause.
TWO_LAUNCH = [(256, 256, 0, 0), (256, 2048, 0, 0), (512, 8192, 0, 0)]


def to_dev(b, status=True):
    bufs = {"x": dev(b.x), "y": dev(b.y), "sd": dev(b.sd), "ed": dev(b.ed),
            "koff": dev(b.koff, torch.int64), "qoff": dev(b.qoff, torch.int64),
            "yq": torch.full((int(b.qoff[-1]),), np.nan, dtype=torch.float64, device="cuda"),
            "ypp": torch.full((int(b.koff[-1]),), np.nan, dtype=torch.float64, device="cuda")}
    st = torch.full((b.count,), 99, dtype=torch.int32, device="cuda") if status else None
    return bufs, st


def check_batch(b, yq, ypp, o=None, what=""):
    if o is None:
        o = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
    o_yq, o_ypp, o_st, _ = o
    assert np.all(o_st == 0)
    for i in range(b.count):
        k0, k1 = b.koff[i], b.koff[i + 1]
        q0, q1 = b.qoff[i], b.qoff[i + 1]
        assert_close(ypp[k0:k1], o_ypp[k0:k1], "%s ypp inst %d" % (what, i))
        assert_close(yq[q0:q1], o_yq[q0:q1], "%s yq inst %d" % (what, i))
    return o


@pytest.fixture(scope="module")
def small_batch():
    return w.batch(seed=3, count=300)


@pytest.fixture(scope="module")
def small_batch_oracle(small_batch):
    b = small_batch
    return oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)


@pytest.mark.parametrize("tuning", TUNINGS + [pytest.param(t, marks=pytest.mark.skip(
    reason="two-launch form removed: it faulted the GPU (memory aperture violation) with no cause found"))
    for t in TWO_LAUNCH])
def test_batch_matches_oracle(small_batch, small_batch_oracle, tuning):
    b = small_batch
    plan = api.spline_plan_create(b.koff, b.qoff, tuning=api.Tuning(*tuning))
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    assert np.all(host(st) == 0)
    check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), small_batch_oracle, "tuning %s" % (tuning,))


def test_batch_mixed_sizes_up_to_limit():
    # curves of every build kind: one per wavefront (n <= 512) and whole
    # workgroup (up to the batch limit), ragged query counts
    n = np.array([3, 4, 5, 13, 64, 65, 511, 512, 513, 1000, 2047, api.MAX_N_BATCH, 3, 130], dtype=np.int64)
    m = np.array([1, 2, 3, 2048, 1023, 1025, 7, 4096, 1, 50000, 333, 2049, 100000, 17], dtype=np.int64)
    b = w.batch_from_sizes(17, n, m)
    for t in ((64, 1024, 1, 1), (256, 4096, 0, 1), (128, 64, 0, 1), (256, 4096, 0, 2), (64, 64, 3, 2)):
        plan = api.spline_plan_create(b.koff, b.qoff, tuning=api.Tuning(*t))
        bufs, st = to_dev(b)
        api.spline_plan_run(plan, bufs, st)
        check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), what="mixed %s" % (t,))


@pytest.mark.parametrize("cap", [64, 1024, 1 << 20])
@pytest.mark.parametrize("fused", [1, 2, 3, 4])
def test_batch_halo_blocks_worst_decay(cap, fused):
    # curves past one wavefront's rows are cut into knot blocks with halos;
    # alternating widths 1 and 1e-3 give the slowest decay of the dropped
    # coupling, and query shares of 64 cut every block many times over
    rng = np.random.default_rng(23)
    sizes = [(api.MAX_N_BATCH, 300000), (1500, 777), (600, 90000), (513, 5)]
    xs, ys = [], []
    for n, _ in sizes:
        x, y = w.alternating_curve(rng, n)
        xs.append(x)
        ys.append(y)
    koff = np.concatenate([[0], np.cumsum([n for n, _ in sizes])]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum([m for _, m in sizes])]).astype(np.int64)
    b = w.Batch(koff, qoff, np.concatenate(xs), np.concatenate(ys), np.array([1e32, 0.0, -1.0, 1e32]),
                np.array([1e32, 0.0, 1.0, 2.0]))
    plan = api.spline_plan_create(b.koff, b.qoff, tuning=api.Tuning(256 if fused >= 3 else 128, cap, 0, fused))
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    assert np.all(host(st) == 0)
    check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), what="halo cap %d" % cap)


def test_batch_single_instance_equals_plain_sizes():
    b = w.batch_from_sizes(5, np.array([13]), np.array([2048]))
    plan = api.spline_plan_create(b.koff, b.qoff)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), what="single")


@pytest.mark.parametrize("fused", [1, 2, 3, 4])
def test_batch_invalid_instance_flags_status(fused):
    b = w.batch(seed=4, count=40)
    x = b.x.copy()
    bad = 7
    x[b.koff[bad] + 1] = x[b.koff[bad]]          # repeated knot in curve 7
    b2 = w.Batch(b.koff, b.qoff, x, b.y, b.sd, b.ed)
    plan = api.spline_plan_create(b2.koff, b2.qoff, tuning=api.Tuning(256, 4096, 0, fused))
    bufs, st = to_dev(b2)
    api.spline_plan_run(plan, bufs, st)
    s = host(st)
    assert s[bad] == api.E_ORDER
    assert np.all(np.delete(s, bad) == 0)
    ypp = host(bufs["ypp"])
    assert np.all(np.isnan(ypp[b.koff[bad]:b.koff[bad + 1]]))
    assert np.all(np.isnan(host(bufs["yq"])[b.qoff[bad]:b.qoff[bad + 1]]))


def test_plan_rejects_bad_sizes():
    with pytest.raises(api.SolveError) as e:
        api.spline_plan_create([0, 2], [0, 10])
    assert e.value.code == api.E_SIZE
    with pytest.raises(api.SolveError) as e:
        api.spline_plan_create([0, api.MAX_N_BATCH + 1], [0, 10])
    assert e.value.code == api.E_SIZE
    with pytest.raises(api.SolveError) as e:
        api.spline_plan_create([0, 5], [0, 0])
    assert e.value.code == api.E_SIZE
    for bad in ((96, 1024, 0, 1), (512, 1024, 0, 1), (128, 1024, 0, 0), (256, 32, 0, 1), (256, 1024, -1, 1),
                (256, 1024, 0, 5), (64, 1024, 0, 3), (128, 1024, 0, 4)):
        with pytest.raises(api.SolveError) as e:
            api.spline_plan_create([0, 5], [0, 10], tuning=api.Tuning(*bad))
        assert e.value.code == api.E_ARG


def test_graph_replays_match_eager(small_batch, small_batch_oracle):
    b = small_batch
    plan = api.spline_plan_create(b.koff, b.qoff)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    eager_yq, eager_ypp = host(bufs["yq"]).copy(), host(bufs["ypp"]).copy()
    stream = torch.cuda.Stream()
    api.spline_plan_capture(plan, bufs, st, stream=stream)
    for r in range(4):
        bufs["yq"].fill_(np.nan)
        bufs["ypp"].fill_(np.nan)
        torch.cuda.synchronize()
        api.spline_plan_replay(plan, stream=stream)
        stream.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(bufs["yq"]), eager_yq)
        np.testing.assert_array_equal(host(bufs["ypp"]), eager_ypp)
        assert np.all(host(st) == 0)
    del junk
    check_batch(b, eager_yq, eager_ypp, small_batch_oracle, "graph")


def test_autotune_picks_a_valid_tuning_and_caches(small_batch, small_batch_oracle):
    b = small_batch
    plan = api.spline_plan_create(b.koff, b.qoff)
    bufs, st = to_dev(b)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        best, ms = api.spline_plan_autotune(plan, bufs, reps=3, cache_path=path)
        assert ms > 0
        assert best.fused in (1, 2, 3)
        assert best.block in (64, 128, 256)
        assert os.path.exists(path)
        got = api.spline_plan_get_tuning(plan)
        assert (got.block, got.queries_per_tile, got.grid_per_cu, got.fused) == \
            (best.block, best.queries_per_tile, best.grid_per_cu, best.fused)
        # a second tune hits the cache
        best2, ms2 = api.spline_plan_autotune(plan, bufs, reps=3, cache_path=path)
        assert (best2.block, best2.queries_per_tile, best2.grid_per_cu, best2.fused) == \
            (best.block, best.queries_per_tile, best.grid_per_cu, best.fused)
        assert ms2 == pytest.approx(ms, rel=1e-5)
    api.spline_plan_run(plan, bufs, st)
    check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), small_batch_oracle, "tuned")


def test_full_batched_config():
    b = w.batch(seed=0)
    plan = api.spline_plan_create(b.koff, b.qoff)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    assert np.all(host(st) == 0)
    check_batch(b, host(bufs["yq"]), host(bufs["ypp"]), what="4096 curves")


def test_batch_result_independent_of_company():
    # the same curve alone and inside a batch gives identical bits
    b = w.batch(seed=6, count=64)
    plan = api.spline_plan_create(b.koff, b.qoff)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    all_yq, all_ypp = host(bufs["yq"]), host(bufs["ypp"])
    for i in (0, 5, 63):
        inst = b.instance(i)
        bi = w.Batch(np.array([0, inst.n]), np.array([0, inst.m]), inst.x, inst.y, np.array([inst.start_deriv]),
                     np.array([inst.end_deriv]))
        p1 = api.spline_plan_create(bi.koff, bi.qoff)
        b1, s1 = to_dev(bi)
        api.spline_plan_run(p1, b1, s1)
        np.testing.assert_array_equal(host(b1["yq"]), all_yq[b.qoff[i]:b.qoff[i + 1]])
        np.testing.assert_array_equal(host(b1["ypp"]), all_ypp[b.koff[i]:b.koff[i + 1]])


# Mixed precision (FP32 sweeps, FP64 residual refinement of y'', FP32 cubic
# term of the evaluation around the FP64 linear part).  Bounds, in the
# per-instance scaled metric |g - o| / (|o| + max|o|):
#   y'': one refinement step takes the FP32 solve error (~2^-24 times the
#        conditioning of the diagonally dominant system) to its square,
#        far below 1e-9 (the 4096-curve batch measures 2.1e-14 at most);
#   y_q: the FP32 cubic term carries a few 2^-24 of its own size, which can
#        exceed the values' scale by a small factor: 4e-6 (the 4096-curve
#        batch measures 1.2e-6 at most, 1.4e-7 at the median).
MIXED_YPP_TOL = 1e-9
MIXED_YQ_TOL = 4e-6


def mixed_errors(b, yq, ypp, o):
    from gpu_util import close
    o_yq, o_ypp, _, _ = o
    e_yq, e_ypp = [], []
    for i in range(b.count):
        k0, k1 = b.koff[i], b.koff[i + 1]
        q0, q1 = b.qoff[i], b.qoff[i + 1]
        e_ypp.append(close(ypp[k0:k1], o_ypp[k0:k1])[1])
        e_yq.append(close(yq[q0:q1], o_yq[q0:q1])[1])
    return np.array(e_yq), np.array(e_ypp)


@pytest.mark.parametrize("tuning", [(256, 4096, 0, 2), (64, 1024, 0, 1), (256, 4096, 0, 3)])
def test_mixed_precision_within_stated_error(small_batch, small_batch_oracle, tuning):
    b = small_batch
    plan = api.spline_plan_create(b.koff, b.qoff, precision=api.FP32_REFINE, tuning=api.Tuning(*tuning))
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    assert np.all(host(st) == 0)
    e_yq, e_ypp = mixed_errors(b, host(bufs["yq"]), host(bufs["ypp"]), small_batch_oracle)
    assert e_ypp.max() <= MIXED_YPP_TOL, e_ypp.max()
    assert e_yq.max() <= MIXED_YQ_TOL, e_yq.max()
    # and it is really the FP32 path: the FP64 path is far closer
    assert e_yq.max() > 1e-12


@pytest.mark.parametrize("top", [3, 64, 65, 128, 129, 192, 193, 256, 257, 384, 385, 512, 513])
def test_mixed_precision_each_group_width(top):
    """The lane-parallel FP32 build at each of its widths (1, 2, 3, 4, 6 or 8
    rows per lane of a wavefront, chosen by the batch's longest curve of at
    most 512 knots), every end condition, curves from 3 knots up to the top
    size; with top = 513 one curve goes to the one-lane sweep build and the
    rest to the lane-parallel one."""
    rng = np.random.default_rng(top)
    n = np.concatenate([[3, 4, 5, top, top], rng.integers(3, top + 1, 59)]).astype(np.int64)
    m = rng.integers(1, 3000, len(n)).astype(np.int64)
    b = w.batch_from_sizes(100 + top, n, m)
    o = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
    plan = api.spline_plan_create(b.koff, b.qoff, precision=api.FP32_REFINE)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    assert np.all(host(st) == 0)
    e_yq, e_ypp = mixed_errors(b, host(bufs["yq"]), host(bufs["ypp"]), o)
    assert e_ypp.max() <= MIXED_YPP_TOL, (top, e_ypp.max())
    assert e_yq.max() <= MIXED_YQ_TOL, (top, e_yq.max())


def test_mixed_precision_long_curves_and_bad_knots():
    n = np.array([3, 13, 300, 1000, api.MAX_N_BATCH, 130], dtype=np.int64)
    m = np.array([5, 2048, 40000, 7, 100000, 20480], dtype=np.int64)
    b = w.batch_from_sizes(29, n, m)
    x = b.x.copy()
    x[b.koff[5] + 3] = x[b.koff[5] + 2]  # curve 5: repeated knot
    b = w.Batch(b.koff, b.qoff, x, b.y, b.sd, b.ed)
    o = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
    plan = api.spline_plan_create(b.koff, b.qoff, precision=api.FP32_REFINE)
    bufs, st = to_dev(b)
    api.spline_plan_run(plan, bufs, st)
    s = host(st)
    assert s[5] == api.E_ORDER and np.all(s[:5] == 0)
    yq, ypp = host(bufs["yq"]), host(bufs["ypp"])
    assert np.all(np.isnan(ypp[b.koff[5]:b.koff[6]])) and np.all(np.isnan(yq[b.qoff[5]:b.qoff[6]]))
    good = w.Batch(b.koff[:6], b.qoff[:6], b.x[:b.koff[5]], b.y[:b.koff[5]], b.sd[:5], b.ed[:5])
    og = oracle.batch_uniform(good.koff, good.qoff, good.x, good.y, good.sd, good.ed)
    e_yq, e_ypp = mixed_errors(good, yq[:good.qoff[-1]], ypp[:good.koff[-1]], og)
    assert e_ypp.max() <= MIXED_YPP_TOL and e_yq.max() <= MIXED_YQ_TOL, (e_ypp, e_yq)
