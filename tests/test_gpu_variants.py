"""The evaluation formulas of the paper's "Curve Interpolation" benchmark
(newint with the hoisted reciprocal, newint__orig, newint__noinv,
splint_one__div, splint_one__mul) on the one-launch wavefront kernel: each
matches the FP64 oracle, and the hoisted form is the default path bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, host
from paper_2001_09253_amd import api, workloads as w

pytestmark = pytest.mark.gpu

BCS = [(1e32, 1e32), (0.0, 0.0), (-1.0, 1.0), (1e32, 0.5)]
# dense (interval-major evaluation) and sparse (per-lane walk) densities,
# blocks with a ragged last block, m = 1 and m = 2
CASES = [(3, 5), (3, 1), (4, 2), (13, 2048), (100, 7), (1025, 4096), (4097, 333), (2000, 200000),
         (13000, 2048000), (250, 3000000)]


def run_variant(x, y, sd, ed, m, variant):
    xd, yd = dev(x), dev(y)
    ypp = torch.full_like(xd, np.nan)
    yq = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    st = torch.zeros((1,), dtype=torch.int32, device="cuda")
    api.spline_solve_uniform_variant(xd, yd, sd, ed, m, variant, yq, ypp, st)
    return host(yq), host(ypp), int(host(st)[0])


@pytest.mark.parametrize("n,m", CASES)
@pytest.mark.parametrize("variant", sorted(api.VARIANTS))
def test_variant_matches_oracle(n, m, variant):
    bc = (n + m) % len(BCS)
    sd, ed = BCS[bc]
    x, y = w.paper_curve(np.random.default_rng(11 * n + bc), n)
    g_yq, g_ypp, st = run_variant(x, y, sd, ed, m, api.VARIANTS[variant])
    o_yq, o_ypp = oracle.spline_uniform(x, y, sd, ed, m)
    assert st == api.OK
    assert_close(g_ypp, o_ypp, "%s ypp n=%d" % (variant, n))
    assert_close(g_yq, o_yq, "%s yq n=%d m=%d" % (variant, n, m))


@pytest.mark.parametrize("n,m", [(13, 2048), (2000, 200000), (13000, 2048000)])
def test_hoisted_variant_is_default_dense_path(n, m):
    # at >= 48 queries per interval spline_solve_uniform takes the same kernel
    x, y = w.paper_curve(np.random.default_rng(n), n)
    g_yq, g_ypp, _ = run_variant(x, y, -1.0, 1.0, m, api.NEWINT_HOISTED)
    xd, yd = dev(x), dev(y)
    ypp = torch.empty_like(xd)
    yq = torch.empty(m, dtype=torch.float64, device="cuda")
    api.spline_solve_uniform(xd, yd, -1.0, 1.0, m, yq, ypp)
    np.testing.assert_array_equal(g_yq, host(yq))
    np.testing.assert_array_equal(g_ypp, host(ypp))


def test_variants_agree_to_rounding():
    inst = w.config_large(seed=4, bc=2)
    outs = {v: run_variant(inst.x, inst.y, inst.start_deriv, inst.end_deriv, inst.m, c)[0]
            for v, c in api.VARIANTS.items()}
    ref = outs["newint"]
    for v, o in outs.items():
        assert_close(o, ref, "%s vs newint" % v, rtol=1e-12)


def test_variant_bad_knots_and_args():
    x, y = w.paper_curve(np.random.default_rng(2), 3000)
    x[1500] = x[1499]
    _, _, st = run_variant(x, y, 0.0, 0.0, 300000, api.SPLINT_MUL)
    assert st == api.E_ORDER
    xd = dev(x)
    yq = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(api.SolveError) as e:
        api.spline_solve_uniform_variant(xd, xd, 0.0, 0.0, 10, 7, yq)
    assert e.value.code == api.E_ARG
    with pytest.raises(api.SolveError) as e:
        api.spline_solve_uniform_variant(xd[:2], xd[:2], 0.0, 0.0, 10, 0, yq)
    assert e.value.code == api.E_SIZE
