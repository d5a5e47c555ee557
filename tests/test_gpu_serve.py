"""The request API (solve_create / submit / poll / wait / destroy) on the GPU:
results against the FP64 oracle, the same result alone and inside a mix,
admission under a small HBM budget, error paths, and an open-loop Poisson
replay through both the batched and the plain path."""
import ctypes as C
import threading

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import _native, api, serve, workloads as w

pytestmark = pytest.mark.gpu


def make_reqs(seed, sizes, explicit=()):
    rng = np.random.default_rng(seed)
    out = []
    for r, (n, m) in enumerate(sizes):
        x, y = w.paper_curve(rng, n)
        _, sd, ed = w.bc_for(r)
        xq = None
        if r in explicit:
            xq = rng.uniform(x[0] - 0.5, x[-1] + 0.5, m)
        out.append((x, y, sd, ed, xq, m))
    return out


def expected(req):
    x, y, sd, ed, xq, m = req
    if xq is None:
        return oracle.spline_uniform(x, y, sd, ed, m)
    ypp = oracle.second_derivatives(x, y, sd, ed)
    return oracle.eval_points(x, y, ypp, xq), ypp


def run_all(ctx, reqs, with_ypp=True, device_out=False):
    outs = []
    tickets = []
    for x, y, sd, ed, xq, m in reqs:
        if device_out:
            yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
            ypp = torch.full((len(x),), np.nan, dtype=torch.float64, device="cuda") if with_ypp else None
        else:
            yq = np.full(m, np.nan)
            ypp = np.full(len(x), np.nan) if with_ypp else None
        tickets.append(api.solve_submit(ctx, x, y, sd, ed, xq, m, yq, ypp))
        outs.append((yq, ypp))
    sts = []
    for r, t in enumerate(tickets):
        assert api.solve_wait(ctx, t) != api.PENDING
        _, code = api.solve_ticket_info(ctx, t)
        st = api.solve_poll(ctx, t)
        assert st == api.DONE or code != api.OK, "request %d: %d with code %d" % (r, st, code)
        sts.append((st, code) if st != api.DONE else st)
    res = []
    for yq, ypp in outs:
        if device_out:
            res.append((host(yq), host(ypp) if ypp is not None else None))
        else:
            res.append((yq, ypp))
    return sts, res


SIZES = [(3, 1), (3, 2048), (4, 5), (13, 2048), (64, 100000), (130, 20480), (257, 3000), (512, 40000),
         (513, 7), (1300, 204800), (api.MAX_N_BATCH, 5000), (40, 1), (700, 90), (13, 205)]


@pytest.mark.parametrize("flags", [0, api.NO_GRAPH])
def test_requests_match_oracle(flags):
    reqs = make_reqs(1, SIZES, explicit={2, 6, 12})
    ctx = api.solve_create(flags=flags)
    try:
        sts, res = run_all(ctx, reqs)
    finally:
        api.solve_destroy(ctx)
    for r, (req, st, (yq, ypp)) in enumerate(zip(reqs, sts, res)):
        assert st == api.DONE, r
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "request %d ypp" % r)
        assert_close(yq, o_yq, "request %d yq" % r)


@pytest.mark.parametrize("explicit", ["all", "every_third"])
def test_explicit_points_share_one_launch(explicit):
    """Requests with explicit points are evaluated together, one launch per
    batch, after the batch is reordered so that they come last: every
    request explicit, and every third (the reordering moves the others)."""
    sizes = SIZES * 2
    ex = set(range(len(sizes))) if explicit == "all" else set(range(0, len(sizes), 3))
    reqs = make_reqs(30, sizes, explicit=ex)
    ctx = api.solve_create()
    try:
        sts, res = run_all(ctx, reqs)
        stats = api.solve_stats(ctx)
    finally:
        api.solve_destroy(ctx)
    assert stats["completed"] == len(reqs)
    for r, (req, st, (yq, ypp)) in enumerate(zip(reqs, sts, res)):
        assert st == api.DONE, r
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "request %d ypp" % r)
        assert_close(yq, o_yq, "request %d yq" % r)


def test_device_outputs_and_device_inputs():
    reqs = make_reqs(2, SIZES[:8])
    ctx = api.solve_create()
    try:
        # device-resident inputs as well
        dreqs = [(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(), sd, ed, xq, m) for x, y, sd, ed, xq, m in reqs]
        sts, res = run_all(ctx, dreqs, device_out=True)
    finally:
        api.solve_destroy(ctx)
    for r, (req, st, (yq, ypp)) in enumerate(zip(reqs, sts, res)):
        assert st == api.DONE
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "request %d ypp" % r)
        assert_close(yq, o_yq, "request %d yq" % r)


def test_pinned_host_outputs():
    reqs = make_reqs(13, SIZES, explicit={2})
    ctx = api.solve_create()
    try:
        outs, tickets = [], []
        for x, y, sd, ed, xq, m in reqs:
            yq = torch.full((m,), np.nan, dtype=torch.float64, pin_memory=True)
            ypp = torch.full((len(x),), np.nan, dtype=torch.float64, pin_memory=True)
            tickets.append(api.solve_submit(ctx, x, y, sd, ed, xq, m, yq, ypp))
            outs.append((yq, ypp))
        for t in tickets:
            api.solve_wait(ctx, t)
            assert api.solve_poll(ctx, t) == api.DONE
    finally:
        api.solve_destroy(ctx)
    for r, (req, (yq, ypp)) in enumerate(zip(reqs, outs)):
        o_yq, o_ypp = expected(req)
        assert_close(ypp.numpy(), o_ypp, "pinned ypp %d" % r)
        assert_close(yq.numpy(), o_yq, "pinned yq %d" % r)


def test_result_same_alone_and_in_the_mix():
    reqs = make_reqs(3, SIZES, explicit={6})
    ctx = api.solve_create(max_inflight=1)
    try:
        _, mix = run_all(ctx, reqs)
        alone = []
        for req in reqs:
            _, one = run_all(ctx, [req])
            alone.append(one[0])
    finally:
        api.solve_destroy(ctx)
    for r in range(len(reqs)):
        np.testing.assert_array_equal(alone[r][0], mix[r][0], "request %d yq" % r)
        np.testing.assert_array_equal(alone[r][1], mix[r][1], "request %d ypp" % r)


def test_plain_path_matches_oracle_and_batched():
    reqs = make_reqs(4, SIZES, explicit={2})
    ctx = api.solve_create(flags=api.PLAIN)
    try:
        sts, res = run_all(ctx, reqs)
    finally:
        api.solve_destroy(ctx)
    for r, (req, st, (yq, ypp)) in enumerate(zip(reqs, sts, res)):
        assert st == api.DONE
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "plain request %d ypp" % r)
        assert_close(yq, o_yq, "plain request %d yq" % r)


def test_plain_path_takes_curves_past_the_batch_limit():
    reqs = make_reqs(5, [(api.MAX_N_BLOCK, 100000), (5000, 3)])
    ctx = api.solve_create(flags=api.PLAIN)
    try:
        sts, res = run_all(ctx, reqs)
    finally:
        api.solve_destroy(ctx)
    for req, st, (yq, ypp) in zip(reqs, sts, res):
        assert st == api.DONE
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "plain ypp")
        assert_close(yq, o_yq, "plain yq")


@pytest.mark.parametrize("flags", [0, api.NO_GRAPH, api.PLAIN])
def test_long_curves_through_the_request_api(flags):
    # curves past the batched kernels' limit (up to 2^20 knots here) take the
    # single-curve kernels, alone (plain) or beside batched requests
    sizes = [(1 << 20, 1 << 20), (13, 2048), ((1 << 20) + 5, 100000), (api.MAX_N_BATCH + 1, 3000), (200, 5000),
             (300000, 7)]
    reqs = make_reqs(21, sizes, explicit={2})
    ctx = api.solve_create(flags=flags)
    try:
        sts, res = run_all(ctx, reqs)
    finally:
        api.solve_destroy(ctx)
    for r, (req, st, (yq, ypp)) in enumerate(zip(reqs, sts, res)):
        assert st == api.DONE, r
        o_yq, o_ypp = expected(req)
        assert_close(ypp, o_ypp, "long request %d ypp" % r)
        assert_close(yq, o_yq, "long request %d yq" % r)


def delay(t, reps=40):
    """Queue about a few milliseconds of work on the current stream."""
    for _ in range(reps):
        t.mul_(1.0)


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("own_stream", [False, True])
def test_device_io_ordered_after_the_callers_stream(plain, own_stream):
    # The knots and values are produced, and the outputs cleared, by work
    # queued on the caller's stream just before solve_submit, behind a few
    # milliseconds of other work: the library reads the inputs after it (the
    # zeros there before would be refused as unordered knots) and writes the
    # results after the clearing fill.
    reqs = make_reqs(22, [(513, 40000), (13, 2048), (3000, 5000)], explicit={2})
    s = torch.cuda.Stream() if own_stream else torch.cuda.default_stream()
    ballast = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
    srcs = [(dev(x), dev(y), dev(xq) if xq is not None else None) for x, y, _, _, xq, _ in reqs]
    torch.cuda.synchronize()
    ctx = api.solve_create(flags=api.PLAIN if plain else 0, stream=s if own_stream else None)
    try:
        outs, tickets = [], []
        for (x, y, sd, ed, xq, m), (sx, sy, sq) in zip(reqs, srcs):
            xd = torch.zeros_like(sx)
            yd = torch.zeros_like(sy)
            qd = torch.zeros_like(sq) if sq is not None else None
            yq = torch.zeros(m, dtype=torch.float64, device="cuda")
            ypp = torch.zeros_like(sx)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                delay(ballast)
                xd.copy_(sx)
                yd.copy_(sy)
                if qd is not None:
                    qd.copy_(sq)
                yq.fill_(-7.0)
                ypp.fill_(-7.0)
                tickets.append(api.solve_submit(ctx, xd, yd, sd, ed, qd, m, yq, ypp))
            outs.append((yq, ypp, xd, yd, qd))
        for t in tickets:
            assert api.solve_wait(ctx, t) == api.DONE
            assert api.solve_poll(ctx, t) == api.DONE
    finally:
        api.solve_destroy(ctx)
    for r, (req, (yq, ypp, *_)) in enumerate(zip(reqs, outs)):
        o_yq, o_ypp = expected(req)
        assert_close(host(ypp), o_ypp, "ordered ypp %d" % r)
        assert_close(host(yq), o_yq, "ordered yq %d" % r)


def test_admission_under_a_small_budget():
    sizes = [(int(n), int(m)) for n, m in zip(*w.log_uniform_sizes(np.random.default_rng(6), 120, 0.1, 10))]
    reqs = make_reqs(6, sizes)
    biggest = max(8 * (3 * n + m) + 64 for n, m in sizes)
    budget = 3 * biggest
    ctx = api.solve_create(hbm_budget_bytes=budget, max_inflight=2)
    try:
        sts, res = run_all(ctx, reqs)
        stats = api.solve_stats(ctx)
        mem = api.solve_memory(ctx)
    finally:
        api.solve_destroy(ctx)
    assert all(s == api.DONE for s in sts)
    assert stats["completed"] == len(reqs)
    assert stats["peak_resident_bytes"] <= budget
    assert stats["batches"] > 1
    # the device buffers the slots held: within the budget, but for spare
    # capacity a running batch took while there was room (half its buffers)
    assert 0 < mem["peak_device_bytes"] <= budget + budget // 2
    for r in (0, 17, 60, 119):
        o_yq, o_ypp = expected(reqs[r])
        assert_close(res[r][0], o_yq, "budget yq %d" % r)


@pytest.mark.parametrize("flags", [0, api.PLAIN])
def test_device_memory_within_the_budget(flags):
    # many small requests (the slots' buffers grow with spare capacity while
    # the budget has room), then large ones that need the room: idle slots
    # give theirs up and the buffers are sized exactly
    small = [(13, 2048)] * 40
    large = [(1300, 204800)] * 6 + [(700, 90)] * 3
    reqs = make_reqs(11, small + large)
    big = 8 * (3 * 1300 + 204800)
    budget = 3 * big
    ctx = api.solve_create(hbm_budget_bytes=budget, max_inflight=3, flags=flags)
    try:
        sts, res = run_all(ctx, reqs[:40])
        mem_small = api.solve_memory(ctx)
        sts2, res2 = run_all(ctx, reqs[40:])
        mem = api.solve_memory(ctx)
    finally:
        api.solve_destroy(ctx)
    assert all(s == api.DONE for s in sts + sts2)
    assert 0 < mem_small["device_bytes"] <= budget
    assert mem["peak_device_bytes"] <= budget + budget // 2
    assert mem["device_bytes"] <= budget + budget // 2
    for r in (0, 39, 40, 45, 48):
        o_yq, o_ypp = expected(reqs[r])
        got = (res + res2)[r]
        assert_close(got[0], o_yq, "memory yq %d" % r)
        assert_close(got[1], o_ypp, "memory ypp %d" % r)


@pytest.mark.parametrize("flags", [0, api.PLAIN])
def test_concurrent_submitters(flags):
    # four host threads submit and wait on one context at once (the ctypes
    # calls release the interpreter lock); every result is the oracle's
    rng = np.random.default_rng(41)
    sizes = [(int(n), int(m)) for n, m in zip(rng.integers(3, 3000, 160), rng.integers(1, 60000, 160))]
    reqs = make_reqs(41, sizes, explicit=set(range(0, 160, 9)))
    outs = [None] * len(reqs)
    errors = []
    ctx = api.solve_create(flags=flags, max_inflight=3)

    def worker(w):
        try:
            mine = list(range(w, len(reqs), 4))
            tickets = []
            for r in mine:
                x, y, sd, ed, xq, m = reqs[r]
                yq, ypp = np.full(m, np.nan), np.full(len(x), np.nan)
                tickets.append(api.solve_submit(ctx, x, y, sd, ed, xq, m, yq, ypp))
                outs[r] = (yq, ypp)
            for t in tickets:
                assert api.solve_wait(ctx, t) == api.DONE
                assert api.solve_poll(ctx, t) == api.DONE
        except Exception as e:  # reported by the main thread
            errors.append(e)

    try:
        threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        stats = api.solve_stats(ctx)
    finally:
        api.solve_destroy(ctx)
    assert not errors, errors
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    for r in range(len(reqs)):
        o_yq, o_ypp = expected(reqs[r])
        assert_close(outs[r][1], o_ypp, "concurrent ypp %d" % r)
        assert_close(outs[r][0], o_yq, "concurrent yq %d" % r)


def test_slot_limit_and_continuous_batching():
    sizes = [(13, 2048)] * 300
    reqs = make_reqs(7, sizes)
    ctx = api.solve_create(max_slots=16, max_inflight=2)
    try:
        sts, res = run_all(ctx, reqs, with_ypp=False)
        stats = api.solve_stats(ctx)
    finally:
        api.solve_destroy(ctx)
    assert all(s == api.DONE for s in sts)
    assert stats["peak_batch"] <= 16
    assert stats["batches"] >= 300 // 16
    o_yq, _ = expected(reqs[123])
    assert_close(res[123][0], o_yq, "slot-limited yq")


def test_submit_errors():
    ctx = api.solve_create(hbm_budget_bytes=1 << 20)
    try:
        x = np.linspace(0, 1, 10)
        y = np.sin(x)
        out = np.empty(100)
        with pytest.raises(api.SolveError) as e:
            api.solve_submit(ctx, x[::-1].copy(), y, 1e32, 1e32, None, 100, out)
        assert e.value.code == api.E_ORDER
        with pytest.raises(api.SolveError) as e:
            api.solve_submit(ctx, x[:2].copy(), y[:2].copy(), 1e32, 1e32, None, 100, out)
        assert e.value.code == api.E_SIZE
        with pytest.raises(api.SolveError) as e:
            api.solve_submit(ctx, x, y, 1e32, 1e32, None, 0, out)
        assert e.value.code == api.E_SIZE
        # past the largest curve (checked before any input is read)
        t = C.c_uint64()
        rc = _native.lib().solve_submit(ctx, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data),
                                        api.MAX_N_SOLVE + 1, 1e32, 1e32, None, 10, C.c_void_p(out.ctypes.data),
                                        None, C.byref(t))
        assert rc == api.E_SIZE
        huge = np.empty(1 << 18)
        with pytest.raises(api.SolveError) as e:
            api.solve_submit(ctx, x, y, 1e32, 1e32, None, 1 << 18, huge)
        assert e.value.code == api.E_BUDGET
        t = api.solve_submit(ctx, x, y, 1e32, 1e32, None, 100, out)
        assert api.solve_wait(ctx, t) == api.DONE
        assert api.solve_poll(ctx, t) == api.DONE
        with pytest.raises(api.SolveError) as e:
            api.solve_poll(ctx, t)
        assert e.value.code == api.E_TICKET
        with pytest.raises(api.SolveError) as e:
            api.solve_ticket_info(ctx, 987654321)
        assert e.value.code == api.E_TICKET
    finally:
        api.solve_destroy(ctx)
    with pytest.raises(api.SolveError) as e:
        api.solve_create(hbm_budget_bytes=0)
    assert e.value.code == api.E_ARG


def test_injected_fault_fails_one_batch_only():
    reqs = make_reqs(8, [(13, 2048)] * 4)
    ctx = api.solve_create(max_inflight=1)
    try:
        api.solve_inject_fault(ctx)
        sts, _ = run_all(ctx, reqs[:1])
        assert sts == [(api.ERROR, api.E_DEVICE)]
        sts, res = run_all(ctx, reqs[1:])
        assert sts == [api.DONE] * 3
        o_yq, _ = expected(reqs[2])
        assert_close(res[1][0], o_yq, "after fault")
        stats = api.solve_stats(ctx)
        assert stats["failed"] == 1 and stats["resident_bytes"] == 0
    finally:
        api.solve_destroy(ctx)


def test_destroy_with_work_in_flight():
    reqs = make_reqs(9, [(130, 20480)] * 200)
    outs = [np.empty(20480) for _ in reqs]
    ctx = api.solve_create(max_slots=8, max_inflight=2)
    for (x, y, sd, ed, xq, m), o in zip(reqs, outs):
        api.solve_submit(ctx, x, y, sd, ed, xq, m, o)
    api.solve_destroy(ctx)  # cancels what is queued, drains what is running


def test_ticket_times_are_ordered():
    reqs = make_reqs(10, [(13, 2048)] * 8)
    ctx = api.solve_create()
    try:
        outs = [np.empty(m) for *_, m in reqs]  # must outlive the requests
        ts = [api.solve_submit(ctx, x, y, sd, ed, xq, m, o) for (x, y, sd, ed, xq, m), o in zip(reqs, outs)]
        for t in ts:
            api.solve_wait(ctx, t)
            times, code = api.solve_ticket_info(ctx, t)
            assert code == api.OK
            assert 0 < times[0] <= times[1] <= times[2] <= times[3] <= api.solve_clock()
            api.solve_poll(ctx, t)
    finally:
        api.solve_destroy(ctx)


@pytest.mark.parametrize("plain", [False, True])
def test_poisson_replay_matches_oracle(plain):
    trace = w.poisson_trace(11, rate=2000.0, duration=0.25, lo=0.1, hi=10.0)
    reqs = serve.make_requests(trace, 12)
    res, outs = serve.replay(trace, reqs, plain=plain, keep_outputs=True, pool=64)
    assert res.errors == 0 and res.requests == len(reqs)
    assert np.all(res.latency_s > 0)
    for r in range(0, len(reqs), 7):
        q = reqs[r]
        o_yq, _ = oracle.spline_uniform(q.x, q.y, q.sd, q.ed, q.m)
        assert_close(outs[r], o_yq, "replay request %d" % r)
