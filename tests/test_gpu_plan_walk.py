"""Every index the batched kernels form from a plan's work tables, walked on
the host (no kernel runs): the 4096-curve batch with each tuning form and in
mixed precision, and a batch at the largest batched curve (2048 knots).

The plan is created on the device (its tables are built by the library's
planner and read back with spline_plan_get_tables); the walk then restates,
item by item, what the wave-item and cooperative-item kernels do with an
item: the span they solve or stage, the LDS rows that holds, the interval
constants and first-query tables they fill, and the output range they write,
and checks each against the array it indexes."""
import numpy as np
import pytest

from paper_2001_09253_amd import _native, api, workloads as w

pytestmark = pytest.mark.gpu

HALO = 128           # halo rows on either side of a knot block
LANE_BUILD_MAX = 256  # curves up to this many knots are built by the first launch (tuning fused = 2)
MIXED_WAVE_MAX = 512  # mixed precision: curves up to this many knots take the lane-parallel build
GROUP_LANES = 16


def walk(koff, qoff, precision, tuning):
    count = len(koff) - 1
    n = np.diff(koff)
    m = np.diff(qoff)
    plan = api.spline_plan_create(koff, qoff, precision=precision, tuning=_native.Tuning(*tuning) if tuning else None)
    items, lane, rows = api.spline_plan_get_tables(plan)
    t = api.spline_plan_get_tuning(plan)
    plan.destroy()
    assert rows in (64, 128, 192, 256, 512)
    ch = rows // 64
    # the first launch builds the curves of up to LANE_BUILD_MAX knots with
    # tuning fused = 2 (16 lanes per curve), every curve in mixed precision:
    # those past MIXED_WAVE_MAX knots one wavefront each with the sweeps on one
    # lane (LDS arrays of MAX_N_BATCH rows), the others one wavefront each with
    # the rows spread over its lanes (LDS arrays of 64 CH rows, CH <= 8)
    mixed = precision == api.FP32_REFINE
    prebuilt = api.MAX_N_BATCH if mixed else LANE_BUILD_MAX if t.fused == 2 else 0
    assert sorted(lane.tolist()) == [i for i in range(count) if n[i] <= prebuilt]
    if len(lane):
        assert np.all(np.diff(n[lane]) <= 0), "first-launch curves are sorted by length"
        if mixed:
            grouped = n[lane][n[lane] <= MIXED_WAVE_MAX]
            assert n[lane].max() <= api.MAX_N_BATCH
            # the long ones lead the list: the one-lane launch takes slots
            # 0 .. n_long - 1, the lane-parallel launch the rest
            n_long = int(np.count_nonzero(n[lane] > MIXED_WAVE_MAX))
            assert np.all(n[lane][:n_long] > MIXED_WAVE_MAX) and np.all(n[lane][n_long:] <= MIXED_WAVE_MAX)
        else:
            grouped = n[lane][n[lane] <= LANE_BUILD_MAX]
        if len(grouped) and mixed:
            ch = -(-int(grouped.max()) // 64)
            ch = ch if ch <= 4 else 6 if ch <= 6 else 8  # the widths compiled
            assert grouped.max() <= 64 * ch <= 64 * 8  # the wavefront's LDS rows
        elif len(grouped):
            lane_ch = 4 if grouped.max() <= GROUP_LANES * 4 else 9 if grouped.max() <= GROUP_LANES * 9 else 16
            assert grouped.max() <= GROUP_LANES * lane_ch  # the group's LDS rows (16 CH + 2)
    # item fields against the offsets
    inst = items["inst"].astype(np.int64)
    assert np.all((inst >= 0) & (inst < count))
    assert np.array_equal(items["ko"], koff[inst]) and np.array_equal(items["qo"], qoff[inst])
    assert np.array_equal(items["n"], n[inst]) and np.array_equal(items["m"], m[inst])
    j0 = items["j0"].astype(np.int64)
    j1 = items["j1"].astype(np.int64)
    ni = n[inst]
    assert np.all((j0 >= 0) & (j0 < j1) & (j1 <= ni - 1))
    assert np.all((items["S"] >= 1) & (items["s"] >= 0) & (items["s"] < items["S"]))
    # the span an item solves (BUILD) or stages (first-launch curves) fits
    # the wavefront's rows, and everything indexed in its LDS fits
    built = ni > prebuilt
    whole = (j0 == 0) & (j1 == ni - 1)
    rs = np.where(whole, 0, np.maximum(0, j0 - HALO))
    re = np.where(whole, ni, np.minimum(ni, j1 + 1 + HALO))
    span = np.where(built, re - rs, j1 - np.maximum(j0 - 1, 0) + 1)
    assert np.all(span[built] <= rows), "a solved span exceeds the wavefront's rows"
    assert np.all(span[~built] <= rows + 1), "a staged block exceeds the LDS rows"
    lo = np.where(built, np.maximum(rs - 1, 0), np.maximum(j0 - 1, 0))
    hi = np.where(built, np.minimum(re, ni - 1), j1)
    assert np.all((lo >= 0) & (hi <= ni - 1) & (hi - lo + 1 <= rows + 2)), "staged knots outside the curve or LDS"
    # 1/(b - a) per interval and the first-query table (nt + 1 <= j1 - j0 + 1 entries)
    assert np.all(j1 - j0 <= rows), "interval table beyond the LDS rows"
    # y'' rows of the block [j0, j1] held at so[j - rs]: inside the solved span
    rs_eff = np.where(built, rs, j0)
    assert np.all((j0 - rs_eff >= 0) & (j1 - rs_eff <= rows + 1))
    # every curve's intervals are covered by its blocks exactly once, each
    # block by shares 0 .. S-1 exactly once
    for i in range(count):
        sel = inst == i
        if not sel.any():
            assert n[i] <= prebuilt and m[i] == 0
            continue
        blocks = sorted(set(zip(j0[sel].tolist(), j1[sel].tolist())))
        assert blocks[0][0] == 0 and blocks[-1][1] == n[i] - 1
        for (a0, a1), (b0, _) in zip(blocks, blocks[1:]):
            assert a1 == b0
        for a0, a1 in blocks:
            bs = sel & (j0 == a0) & (j1 == a1)
            S = items["S"][bs]
            assert np.all(S == S[0]) and sorted(items["s"][bs].tolist()) == list(range(S[0]))
    # the queries' output range of each item lies in its curve's (the kernels
    # clamp the block's first and last query into [0, m])
    assert np.all(items["qo"] + items["m"] <= qoff[-1])
    # int16 interval indices hold the batched limit
    assert n.max() <= 32767
    return len(items), ch


CONFIGS = [(api.FP64, None), (api.FP64, (256, 8192, 0, 1)), (api.FP64, (64, 2048, 16, 1)),
           (api.FP64, (256, 4096, 0, 2)), (api.FP64, (256, 16384, 0, 3)), (api.FP64, (256, 8192, 0, 4)),
           (api.FP32_REFINE, None)]


@pytest.mark.parametrize("precision,tuning", CONFIGS)
def test_walk_batched_4096(precision, tuning):
    b = w.batch(seed=0)
    nitems, _ = walk(b.koff, b.qoff, precision, tuning)
    assert nitems >= b.count


@pytest.mark.parametrize("precision,tuning", CONFIGS)
def test_walk_batched_at_the_size_limit(precision, tuning):
    # curves at the batched limit (2048 knots: knot blocks with halos, the
    # widest spans) beside short ones and one-query curves
    rng = np.random.default_rng(3)
    n = np.concatenate([[api.MAX_N_BATCH] * 20, rng.integers(513, api.MAX_N_BATCH, 30), rng.integers(3, 600, 50),
                        [3, 4, 256, 257, 512]])
    m = np.concatenate([rng.integers(1, 300000, 100), [1, 2, 7, 1, 100000]])
    koff = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    walk(koff, qoff, precision, tuning)
