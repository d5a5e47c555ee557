"""The two-level search of the explicit-query kernel, restated on the host and
checked against the definition of the interval (section 2: the interval of q
is the last knot interval starting below q, clipped to the first and last
interval), by brute force.

The kernel keeps every stride-th knot as a fence (at most 8192 fences,
stride = ceil(n / 8192)); with c fences below q, every knot below index
(c - 1) * stride + 1 is below q and none from c * stride on is, so a lower
bound over that one stretch of knots completes the count. A tile of queries
whose smallest and largest query fall in intervals ilo .. ihi with
ihi - ilo + 2 <= 512 stages knots ilo .. ihi + 1 and searches only their
interior. Both are restated here with the kernel's constants and compared
with np.searchsorted over the whole knot vector, for knot counts around the
fence and window boundaries, with queries on knots, one ulp either side,
outside the range, infinite and NaN."""
import math

import numpy as np
import pytest

FENCE_MAX = 8192
WIN = 512


def lower_bound(arr, lo, length, q):
    """First index in arr[lo .. lo + length) whose value is not below q
    (lo + length if none), by bisection; NaN compares false, as on the GPU."""
    while length > 0:
        half = length >> 1
        if arr[lo + half] < q:
            lo, length = lo + half + 1, length - half - 1
        else:
            length = half
    return lo


def clip_interval(cnt, n):
    return min(max(cnt - 1, 0), n - 2)


def geometry(n):
    stride = max(1, (n + FENCE_MAX - 1) // FENCE_MAX)
    nf = (n + stride - 1) // stride
    return stride, nf


def fenced_count(x, fence, stride, q):
    n = len(x)
    c = lower_bound(fence, 0, len(fence), q)
    if c == 0:
        return 0
    lo = (c - 1) * stride + 1
    hi = min(c * stride, n)
    return lower_bound(x, lo, hi - lo, q)


def truth(x, q):
    # the definition: #{x_j < q}, a NaN query counting no knot
    return clip_interval(int(np.count_nonzero(x < q)), len(x))


def knots(n, rng):
    return np.cumsum(rng.uniform(0.1, 1.0, n)) - 0.5 * n


def queries(x, rng, count):
    lo, hi = x[0], x[-1]
    pick = x[rng.integers(0, len(x), count // 4)]
    return np.concatenate([
        rng.uniform(lo - 1.0, hi + 1.0, count // 2), pick, np.nextafter(pick, np.inf), np.nextafter(pick, -np.inf),
        [lo, hi, lo - 1e300, hi + 1e300, np.inf, -np.inf, np.nan, np.nextafter(lo, -np.inf),
         np.nextafter(hi, np.inf)]])


@pytest.mark.parametrize("n", [3, 4, 5, 64, 2047, 2048, 2049, 8191, 8192, 8193, 13000, 16385, 24577, 100003])
def test_fenced_count_is_the_definition(n):
    rng = np.random.default_rng(n)
    x = knots(n, rng)
    stride, nf = geometry(n)
    assert nf <= FENCE_MAX and (nf - 1) * stride < n <= nf * stride
    fence = x[::stride]
    assert len(fence) == nf
    for q in queries(x, rng, 400):
        assert clip_interval(fenced_count(x, fence, stride, q), n) == truth(x, q), (n, q)


def staged_tile(x, fence, stride, tile):
    """The kernel's tile: intervals of the smallest and largest query (NaN
    ignored by min/max); staged when no query is NaN and the window fits."""
    n = len(x)
    vals = tile[~np.isnan(tile)]
    qmin = vals.min() if len(vals) else math.inf
    qmax = vals.max() if len(vals) else -math.inf
    ilo = clip_interval(fenced_count(x, fence, stride, qmin), n)
    ihi = max(clip_interval(fenced_count(x, fence, stride, qmax), n), ilo)
    staged = not np.isnan(tile).any() and ihi - ilo + 2 <= WIN
    out = []
    for q in tile:
        if staged:
            wx = x[ilo:ihi + 2]
            out.append(ilo + lower_bound(wx, 1, len(wx) - 2, q) - 1)
        else:
            out.append(clip_interval(fenced_count(x, fence, stride, q), n))
    return staged, out


@pytest.mark.parametrize("n", [3, 5, 513, 8193, 100003])
def test_staged_window_is_the_definition(n):
    rng = np.random.default_rng(7 + n)
    x = knots(n, rng)
    stride, _ = geometry(n)
    fence = x[::stride]
    seen = set()
    for trial in range(60):
        # sorted runs (narrow tiles), clustered tiles, tiles across the whole
        # range (not staged), and tiles with a NaN or an infinity
        lo = rng.uniform(x[0] - 2, x[-1] + 2)
        width = rng.choice([0.0, 1.0, 30.0, 400.0, x[-1] - x[0] + 4])
        tile = np.sort(rng.uniform(lo, lo + width, 64))
        if trial % 7 == 3:
            tile[5] = np.nan
        if trial % 11 == 4:
            tile[-1] = np.inf
        if trial % 13 == 5:
            tile[:8] = x[rng.integers(0, n, 8)]
        staged, got = staged_tile(x, fence, stride, tile)
        seen.add(staged)
        assert got == [truth(x, q) for q in tile], (n, trial)
    assert seen == {True, False} or n <= WIN - 2
