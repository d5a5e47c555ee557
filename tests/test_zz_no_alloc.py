"""The batched path without device allocation (spline_batch_run_noalloc,
through the C ABI) against the plan it stands in for (spline_plan_create +
spline_plan_run): the same results bit for bit on the 4096-curve batch, then
on a smaller batch in the next call (the device buffer keeps the last call's
tables), with each tuning form and in mixed precision; tables past the
buffer's size are refused before any device work."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import api, _native, workloads as w

pytestmark = pytest.mark.gpu


def buffers(b):
    return {"x": dev(b.x), "y": dev(b.y), "sd": dev(b.sd), "ed": dev(b.ed), "koff": dev(b.koff, torch.int64),
            "qoff": dev(b.qoff, torch.int64),
            "yq": torch.full((int(b.qoff[-1]),), np.nan, dtype=torch.float64, device="cuda"),
            "ypp": torch.full((int(b.koff[-1]),), np.nan, dtype=torch.float64, device="cuda")}


def run_both(b, precision=api.FP64, tuning=None):
    t = _native.Tuning(*tuning) if tuning else None
    ref = buffers(b)
    st_ref = torch.full((b.count,), 99, dtype=torch.int32, device="cuda")
    plan = api.spline_plan_create(b.koff, b.qoff, precision=precision, tuning=t)
    api.spline_plan_run(plan, ref, st_ref)
    got = buffers(b)
    st = torch.full((b.count,), 99, dtype=torch.int32, device="cuda")
    api.spline_batch_run_noalloc(b.koff, b.qoff, got, precision=precision, tuning=t, status=st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(got["yq"]), host(ref["yq"]))
    np.testing.assert_array_equal(host(got["ypp"]), host(ref["ypp"]))
    np.testing.assert_array_equal(host(st), host(st_ref))
    plan.destroy()
    return host(got["yq"]), host(got["ypp"]), host(st)


def sub_batch(b, count):
    kend, qend = int(b.koff[count]), int(b.qoff[count])
    return w.Batch(koff=b.koff[:count + 1].copy(), qoff=b.qoff[:count + 1].copy(), x=b.x[:kend].copy(),
                   y=b.y[:kend].copy(), sd=b.sd[:count].copy(), ed=b.ed[:count].copy())


def test_noalloc_equals_plan_run_twice():
    b = w.batch(seed=0)
    yq, ypp, st = run_both(b)
    assert np.all(st == api.OK)
    o_yq, o_ypp, _, _ = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
    for i in range(0, b.count, 97):
        assert_close(yq[b.qoff[i]:b.qoff[i + 1]], o_yq[b.qoff[i]:b.qoff[i + 1]], "noalloc yq %d" % i)
        assert_close(ypp[b.koff[i]:b.koff[i + 1]], o_ypp[b.koff[i]:b.koff[i + 1]], "noalloc ypp %d" % i)
    # a second call, smaller: the buffer holds the previous call's tables
    small = sub_batch(w.batch(seed=1), 700)
    yq2, _, st2 = run_both(small)
    assert np.all(st2 == api.OK)
    o_yq2, _, _, _ = oracle.batch_uniform(small.koff, small.qoff, small.x, small.y, small.sd, small.ed)
    assert_close(yq2, o_yq2, "noalloc second call")


@pytest.mark.parametrize("precision,tuning", [(api.FP64, (256, 4096, 0, 2)), (api.FP64, (256, 8192, 0, 3)),
                                              (api.FP64, (256, 8192, 0, 4)), (api.FP64, (64, 2048, 16, 1)),
                                              (api.FP32_REFINE, None)])
def test_noalloc_tunings(precision, tuning):
    b = w.batch(seed=2, count=1500)
    run_both(b, precision, tuning)
    run_both(sub_batch(b, 333), precision, tuning)


def test_noalloc_refuses_oversized_tables():
    # 200,000 one-query curves take 200,000 work items, 9.6 MB of tables
    count = 200000
    koff = np.arange(count + 1, dtype=np.int64) * 3
    qoff = np.arange(count + 1, dtype=np.int64)
    bufs = {"x": torch.zeros(3 * count, dtype=torch.float64, device="cuda"),
            "y": torch.zeros(3 * count, dtype=torch.float64, device="cuda"),
            "sd": torch.zeros(count, dtype=torch.float64, device="cuda"),
            "ed": torch.zeros(count, dtype=torch.float64, device="cuda"),
            "koff": dev(koff, torch.int64), "qoff": dev(qoff, torch.int64),
            "yq": torch.zeros(count, dtype=torch.float64, device="cuda"),
            "ypp": torch.zeros(3 * count, dtype=torch.float64, device="cuda")}
    with pytest.raises(api.SolveError) as e:
        api.spline_batch_run_noalloc(koff, qoff, bufs)
    assert e.value.code == api.E_SIZE
