#!/usr/bin/env python3
"""Benchmark of the spline hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
build (validate, rows, parallel Thomas solve for y'') and evaluate (uniform
queries, bracketing, newint) for every curve of the workload.  The metric is
instance-steps per second, where a step of a curve is one knot update or one
query evaluation, so a pass over a curve with n knots and m queries is n + m
steps.  Inputs are resident in HBM before the timed region starts.

Workloads (--workload):
  batched  (default) 4096 curves, sizes log-uniform 0.1x..10x of the worked
           size (13 knots, 2048 queries), seed 0: one launch per step over
           autotuned work items, the outputs rotated over >= 2 GiB so that
           they go to HBM; beside it (unless --no-context) the single-curve
           kernel on C2 and C2x and a short served run against the plain path
  plain    1 curve, n = 13,000 knots, m = 2,048,000 uniform queries (the
           paper's 13-knot / 2048-point worked size scaled 1000x), seed 0
  small    1 curve, n = 13, m = 2048 (the worked size itself)
  plain2x  1 curve, n = 13,000, m = 2^27 (out of the 256 MB last-level cache)
  points   1 curve, n = 13,000, m = 2^27 explicit queries (random, or
           --sorted), with first and second derivatives: the curve's y''
           built and packed, then spline_eval_points_packed
  batched_points
           the batched workload's 4096 curves, each at its own explicit
           points (as many as its uniform queries, uniform over its range,
           random order): a build-only plan, then spline_batch_eval_points,
           values only, inputs and outputs rotated over >= 2 GiB
  long     1 curve, n = m = 2^28 (the size sweep's largest point: one query
           per interval, the streaming kernel)
  mixed    the batched workload with the FP32 solve + FP64 refinement
  served   Poisson arrivals at 2000 req/s (sizes 0.1x..100x) through the
           request API, continuous batching vs the plain one-request path
  sweep    one curve per size, m = n, sizes 4 .. 2^28 from the paper's size
           formula in shuffled order: solve and noop ns/point per size
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "instances·steps/sec + HBM GB/s %peak; p50/p99 latency (served vs plain)"
UNIT = "instance-steps/s"
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2001_09253_amd", "csrc")


def kernel_source_hash() -> str:
    from paper_2001_09253_amd.profiling import kernel_source_hash as ksh
    return ksh()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(PROFILES, "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get("%s|%s" % (kernel, workload))
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def copy_ceiling(reps=20):
    """Measured device-to-device copy rate of 256 MiB (bytes read + written
    per second): the practical ceiling beside the vendor peak."""
    import torch

    nbytes = 256 << 20
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def add_copy_ceiling(out):
    """Report the dominant kernel's rate against the measured copy rate too."""
    gbs = copy_ceiling()
    out["roofline"]["copy_gbs"] = gbs
    out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / gbs
    return out


def bench_single(args, n, m, workload_name, sd=1e32, ed=1e32, cpu_sample=None):
    import numpy as np
    import torch

    from paper_2001_09253_amd import api, workloads

    inst = workloads.single(0, n, m, bc=0)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(inst.x).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    ypp = torch.empty_like(x)
    yq = torch.empty(m, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    sd, ed = inst.start_deriv, inst.end_deriv
    # the two-launch form (build, then evaluate), timed per kernel for
    # reference (its build takes curves of up to SOLVE_MAX_N_BLOCK knots)
    K = args.steps
    build_ms = eval_ms = None
    if n <= api.MAX_N_BLOCK:
        for _ in range(args.warmup):
            api.spline_build(x, y, sd, ed, ypp)
            api.spline_eval_uniform(x, y, ypp, m, yq)
        ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
        for k in range(K):
            ev2[k][0].record(stream)
            api.spline_build(x, y, sd, ed, ypp)
            ev2[k][1].record(stream)
            api.spline_eval_uniform(x, y, ypp, m, yq)
            ev2[k][2].record(stream)
        torch.cuda.synchronize()
        build_ms = sum(e[0].elapsed_time(e[1]) for e in ev2) / K
        eval_ms = sum(e[1].elapsed_time(e[2]) for e in ev2) / K
    # the timed path: one launch per step (build and evaluate fused); with
    # --variant, the one-launch kernel with one of the paper's evaluation
    # formulas
    # (the launch stream is passed explicitly: looking up torch's current
    # stream on every call costs host time the smallest workload would see)
    sp = stream.cuda_stream
    if args.variant is None:
        def solve():
            api.spline_solve_uniform(x, y, sd, ed, m, yq, ypp, stream=sp)
    else:
        code = api.VARIANTS[args.variant]

        def solve():
            api.spline_solve_uniform_variant(x, y, sd, ed, m, code, yq, ypp, stream=sp)
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    # one event pair around the K back-to-back launches on the launch stream:
    # the average launch duration without per-launch event overhead
    e_begin = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_begin.record(stream)
    for k in range(K):
        solve()
    e_end.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solve_ms = e_begin.elapsed_time(e_end) / K
    step_s = (t1 - t0) / K
    # cold runs: a 1 GiB write before each launch evicts the inputs from the
    # caches (the 256 MB last-level cache included); only the launch is timed
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cold = []
    for _ in range(10):
        flush.fill_(1.0)
        ec0 = torch.cuda.Event(enable_timing=True)
        ec1 = torch.cuda.Event(enable_timing=True)
        ec0.record(stream)
        solve()
        ec1.record(stream)
        torch.cuda.synchronize()
        cold.append(ec0.elapsed_time(ec1))
    del flush
    value = (n + m) / step_s
    # algorithmic bytes per launch of the fused kernel: read x, y (16 n),
    # write y'' (8 n) and write the m results (8 m); the halo rows each
    # workgroup re-reads and the y'' it keeps on chip are not counted
    dom = "solve_uniform" if args.variant is None else "solve_uniform[%s]" % args.variant
    dms = solve_ms
    dbytes = 24.0 * n + 8.0 * m
    achieved = dbytes / (dms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload_name, "instances": 1, "n": n, "m": m, "ends": "natural",
                   "eval_formula": args.variant or "newint (hoisted 1/(b-a))",
                   "seed": 0, "generator": "x_j = x_{j-1} + U(0,1) (0 -> 1e-4), y_j = U(0,1)"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, workload_name),
                     "algorithmic_bytes_per_launch": dbytes, "avg_launch_ms": dms},
        "kernels_ms": {dom: solve_ms, "two_launch_build": build_ms, "two_launch_eval_uniform": eval_ms},
        "cold_ms": {"median": float(np.median(cold)), "max": float(np.max(cold)), "runs": len(cold),
                    "note": "one launch after a 1 GiB write evicts the caches"},
        "points_per_s": m / step_s, "knots_per_s": n / step_s,
        "path_gbs": (24.0 * n + 8.0 * m) / step_s / 1e9,
    }
    out["path_frac_peak"] = out["path_gbs"] / HBM_PEAK_GBS
    if not args.no_cpu_baseline:
        if cpu_sample is None:
            out["cpu_baseline"] = cpu_baseline_single(inst, args.cpu_seconds)
        else:
            # a bounded sample: the curve's first cpu_sample knots, queries
            # at the same density
            k = int(cpu_sample)
            sub = workloads.Instance(inst.x[:k], inst.y[:k], sd, ed, max(2, int(round(m * (k - 1) / (n - 1)))))
            out["cpu_baseline"] = cpu_baseline_single(sub, args.cpu_seconds)
    return out


def cpu_baseline_single(inst, seconds):
    import oracle
    import numpy as np

    n, m = inst.n, inst.m
    # one warm call, then whole-workload repetitions for about `seconds`
    oracle.spline_uniform(inst.x, inst.y, inst.start_deriv, inst.end_deriv, m)
    reps = 0
    t0 = oracle.now()
    while True:
        oracle.spline_uniform(inst.x, inst.y, inst.start_deriv, inst.end_deriv, m)
        reps += 1
        t = oracle.now() - t0
        if t >= seconds:
            break
    per = t / reps
    return {"value": (n + m) / per, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": "whole workload (n=%d, m=%d) repeated %d times in %.1f s, single thread" % (n, m, reps, t),
            "ns_per_point": per / m * 1e9}


def host_cpu():
    """Logical CPUs this process may use and the CPU model name (from lscpu,
    else /proc/cpuinfo)."""
    import subprocess
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        ncpu = os.cpu_count() or 1
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return ncpu, model


def bench_batched(args, precision):
    import numpy as np
    import torch

    from paper_2001_09253_amd import api, workloads

    b = workloads.batch(seed=0)
    bufs = {"x": torch.from_numpy(b.x).cuda(), "y": torch.from_numpy(b.y).cuda(),
            "sd": torch.from_numpy(b.sd).cuda(), "ed": torch.from_numpy(b.ed).cuda(),
            "koff": torch.from_numpy(b.koff).cuda(), "qoff": torch.from_numpy(b.qoff).cuda(),
            "yq": torch.empty(int(b.qoff[-1]), dtype=torch.float64, device="cuda"),
            "ypp": torch.empty(int(b.koff[-1]), dtype=torch.float64, device="cuda")}
    plan = api.spline_plan_create(b.koff, b.qoff, precision=precision)
    cache = os.path.join(ROOT, "paper_2001_09253_amd", "autotune.json")
    best, best_ms = api.spline_plan_autotune(plan, bufs, reps=5, cache_path=cache)
    stream = torch.cuda.Stream()
    api.spline_plan_capture(plan, bufs, stream=stream)
    K = args.steps

    def timed(step):
        # K steps back to back on `stream`, one event pair around them (the
        # average step without per-step event overhead) and the host clock
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        e_begin = torch.cuda.Event(enable_timing=True)
        e_end = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e_begin.record(stream)
        for k in range(K):
            step()
        e_end.record(stream)
        stream.synchronize()
        t1 = time.perf_counter()
        return e_begin.elapsed_time(e_end) / K, (t1 - t0) / K

    # context first: the step as a hipGraph replay and as a direct launch on
    # the same output buffers (which then stay in the 256 MB last-level cache)
    replay_ms, replay_s = timed(lambda: api.spline_plan_replay(plan, stream=stream))
    warm_ms, warm_s = timed(lambda: api.spline_plan_run(plan, bufs, stream=stream))
    # the measured steps, last: direct launches with the outputs rotated over
    # >= 2 GiB, so that no launch finds its outputs in the last-level cache
    # (the results go to HBM, as a job larger than the cache would send them)
    out_bytes = 8 * (int(b.qoff[-1]) + int(b.koff[-1]))
    nrot = max(2, -(-(2 << 30) // out_bytes))
    rot = [dict(bufs, yq=torch.empty_like(bufs["yq"]), ypp=torch.empty_like(bufs["ypp"])) for _ in range(nrot)]
    it = [0]

    def rotated():
        api.spline_plan_run(plan, rot[it[0] % nrot], stream=stream)
        it[0] += 1
    rot_ms, rot_s = timed(rotated)
    del rot
    N, M = int(b.koff[-1]), int(b.qoff[-1])
    value = (N + M) / rot_s
    # algorithmic bytes per launch: read x, y (16 per knot), write y'' (8 per
    # knot) and the results (8 per query), and per curve its two end
    # derivatives and two offsets (8 each) and its 48-byte work item
    dbytes = 24.0 * N + 8.0 * M + 16.0 * b.count * 2 + 8.0 * b.count * 2
    achieved = dbytes / (rot_ms * 1e-3) / 1e9
    wl = "batched" if precision == api.FP64 else "mixed"
    kern = "coop_items" if best.fused == 3 else "wave_items"
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": rot_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == api.FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "%s: 4096 curves, sizes log-uniform 0.1x..10x of (13 knots, 2048 queries), one "
                               "launch per step, outputs rotated over %.1f GB" % (wl, nrot * out_bytes / 1e9),
                   "instances": b.count, "sum_n": N, "sum_m": M, "ends": "natural/flat/twist cycle", "seed": 0,
                   "generator": "x_j = x_{j-1} + U(0,1) (0 -> 1e-4), y_j = U(0,1)",
                   "tuning": {"block": best.block, "queries_per_tile": best.queries_per_tile,
                              "grid_per_cu": best.grid_per_cu, "fused": best.fused}},
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kern, wl),
                     "algorithmic_bytes_per_launch": dbytes, "avg_launch_ms": rot_ms},
        "step_ms": {"outputs_rotated": rot_ms, "host_outputs_rotated": rot_s * 1e3,
                    "outputs_in_cache": warm_ms, "host_outputs_in_cache": warm_s * 1e3,
                    "graph_replay_outputs_in_cache": replay_ms, "host_graph_replay": replay_s * 1e3},
        "outputs_in_cache": {"frac": dbytes / (warm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "note": "the same launch with its outputs left in the last-level cache"},
        "rotated_outputs": {"buffers": nrot, "bytes": nrot * out_bytes},
    }
    if precision != api.FP64:
        # per-instance error of the mixed path against the FP64 oracle, in
        # the scaled metric |g - o| / (|o| + max|o| of the instance)
        import oracle
        api.spline_plan_run(plan, bufs, stream=stream)
        stream.synchronize()
        o_yq, o_ypp, _, _ = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
        yq = bufs["yq"].cpu().numpy()
        ypp = bufs["ypp"].cpu().numpy()

        def scaled(g, o):
            sc = np.max(np.abs(o)) if o.size else 0.0
            return float(np.max(np.abs(g - o) / (np.abs(o) + sc + 1e-300))) if o.size else 0.0

        e_yq = np.array([scaled(yq[b.qoff[i]:b.qoff[i + 1]], o_yq[b.qoff[i]:b.qoff[i + 1]]) for i in range(b.count)])
        e_ypp = np.array([scaled(ypp[b.koff[i]:b.koff[i + 1]], o_ypp[b.koff[i]:b.koff[i + 1]])
                          for i in range(b.count)])
        out["error_vs_oracle"] = {
            "metric": "per instance max |g - o| / (|o| + max|o|)",
            "yq": {"max": float(e_yq.max()), "p50": float(np.median(e_yq)), "p99": float(np.percentile(e_yq, 99))},
            "ypp": {"max": float(e_ypp.max()), "p50": float(np.median(e_ypp)),
                    "p99": float(np.percentile(e_ypp, 99))}}
    if not args.no_cpu_baseline:
        import oracle
        # the oracle over the whole batch (all 4096 curves), OpenMP over
        # curves on the host's cores, repeated for about --cpu-seconds
        ncpu, model = host_cpu()
        t0 = oracle.now()
        reps = 0
        used = 1
        while True:
            _, _, _, used = oracle.batch_uniform(b.koff, b.qoff, b.x, b.y, b.sd, b.ed)
            reps += 1
            if oracle.now() - t0 >= args.cpu_seconds:
                break
        t = oracle.now() - t0
        out["cpu_baseline"] = {"value": (N + M) * reps / t, "unit": UNIT, "cores": used, "kind": "oracle",
                               "sample": "the whole batch (all %d curves), %d repetitions in %.1f s, OpenMP over "
                                         "curves on %d threads" % (b.count, reps, t, used),
                               "nproc": ncpu, "cpu_model": model, "ms_per_step": t / reps * 1e3}
    return out


def bench_points(args, sorted_queries):
    """Explicit queries at scale: one curve of 13,000 knots and 2^27 query
    points drawn uniformly over its range (in random order, or sorted), each
    bracketed by search and evaluated with its first and second derivative.
    A step is the build (y'' of the curve) plus the evaluation of every
    point."""
    import numpy as np
    import torch

    from paper_2001_09253_amd import api, workloads

    n, m = 13000, 1 << 27
    inst = workloads.single(0, n, m, bc=0)
    rng = np.random.default_rng(1)
    xq_h = rng.uniform(inst.x[0], inst.x[-1], m)
    x = torch.from_numpy(inst.x).cuda()
    y = torch.from_numpy(inst.y).cuda()
    xq = torch.from_numpy(xq_h).cuda()
    if sorted_queries:
        xq = torch.sort(xq).values.contiguous()
    ypp = torch.empty_like(x)
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    yq = torch.empty(m, dtype=torch.float64, device="cuda")
    d1 = torch.empty_like(yq)
    d2 = torch.empty_like(yq)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    sd, ed = inst.start_deriv, inst.end_deriv
    K = args.steps

    packed = torch.empty(3 * n, dtype=torch.float64, device="cuda")

    def build():  # y'' of the curve (the single-launch kernel, one throw-away query), then x, y, y'' interleaved
        api.spline_solve_uniform(x, y, sd, ed, 1, one, ypp, stream=sp)
        api.spline_pack_knots(x, y, ypp, packed, stream=sp)

    def evaluate(derivs):
        api.spline_eval_points_packed(packed, xq, yq, d1 if derivs else None, d2 if derivs else None, stream=sp)

    def evaluate_unpacked(derivs):
        api.spline_eval_points(x, y, ypp, xq, yq, d1 if derivs else None, d2 if derivs else None, stream=sp)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(K):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K, (time.perf_counter() - t0) / K

    build_ms, _ = timed(build)
    vals_ms, _ = timed(lambda: evaluate(False))
    eval_ms, _ = timed(lambda: evaluate(True))
    unpacked_vals_ms, _ = timed(lambda: evaluate_unpacked(False))
    unpacked_ms, _ = timed(lambda: evaluate_unpacked(True))
    step_ms, step_s = timed(lambda: (build(), evaluate(True)))
    # algorithmic bytes of the evaluation launch: read the points (8 per
    # query), write value, first and second derivative (24 per query), read
    # x, y and y'' (24 per knot)
    dbytes = 32.0 * m + 24.0 * n
    achieved = dbytes / (eval_ms * 1e-3) / 1e9
    wl = "points_sorted" if sorted_queries else "points"
    out = {
        "metric": METRIC, "value": (n + m) / step_s, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s: 1 curve, n=13000, m=2^27 explicit points (%s), value + first and second "
                               "derivative, from the packed curve" % (wl, "sorted" if sorted_queries else "random order"),
                   "instances": 1, "n": n, "m": m, "ends": "natural", "seed": 0,
                   "points": "U(x_0, x_{n-1}), numpy default_rng(1)"},
        "roofline": {"bound": "hbm", "kernel": "eval_points", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("eval_points", wl),
                     "algorithmic_bytes_per_launch": dbytes, "avg_launch_ms": eval_ms},
        "kernels_ms": {"build_and_pack": build_ms, "eval_points_values": vals_ms,
                       "eval_points_with_derivatives": eval_ms, "unpacked_values": unpacked_vals_ms,
                       "unpacked_with_derivatives": unpacked_ms, "step_event_ms": step_ms},
        "values_only": {"ms": vals_ms, "frac": (16.0 * m + 24.0 * n) / (vals_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        import oracle
        # the oracle, single thread, on the first 2^22 points (value and
        # derivatives), repeated for about --cpu-seconds
        k = 1 << 22
        q = np.ascontiguousarray(np.sort(xq_h[:k]) if sorted_queries else xq_h[:k])
        o_ypp = oracle.second_derivatives(inst.x, inst.y, sd, ed)
        reps = 0
        t0 = oracle.now()
        while True:
            oracle.eval_points(inst.x, inst.y, o_ypp, q)
            oracle.eval_points_derivs(inst.x, inst.y, o_ypp, q)
            reps += 1
            if oracle.now() - t0 >= args.cpu_seconds:
                break
        t = oracle.now() - t0
        out["cpu_baseline"] = {"value": k * reps / t, "unit": UNIT, "cores": 1, "kind": "oracle",
                               "sample": "the first 2^22 points (%s), value and derivatives, %d repetitions in "
                                         "%.1f s, single thread (the build of y'' not timed)"
                                         % ("sorted" if sorted_queries else "random order", reps, t),
                               "ns_per_point": t / (k * reps) * 1e9}
    return out


def bench_batched_points(args):
    """The explicit variant of the batched workload: C3's 4096 curves, each
    evaluated at its own m_i points (uniform over [x_0, x_{n-1}] of the curve,
    random order).  A step is the build of every curve's y'' (a build-only
    plan, one launch) and the evaluation of every point (one launch)."""
    import numpy as np
    import torch

    from paper_2001_09253_amd import api, workloads

    b = workloads.batch(seed=0)
    rng = np.random.default_rng(1)
    xq_h = np.empty(int(b.qoff[-1]))
    for i in range(b.count):
        x = b.x[b.koff[i]:b.koff[i + 1]]
        xq_h[b.qoff[i]:b.qoff[i + 1]] = rng.uniform(x[0], x[-1], int(b.qoff[i + 1] - b.qoff[i]))
    N, M = int(b.koff[-1]), int(b.qoff[-1])
    bufs = {"x": torch.from_numpy(b.x).cuda(), "y": torch.from_numpy(b.y).cuda(),
            "sd": torch.from_numpy(b.sd).cuda(), "ed": torch.from_numpy(b.ed).cuda(),
            "koff": torch.from_numpy(b.koff).cuda(), "ypp": torch.empty(N, dtype=torch.float64, device="cuda")}
    qoff = torch.from_numpy(b.qoff).cuda()
    plan = api.spline_plan_create(b.koff, None)
    cache = os.path.join(ROOT, "paper_2001_09253_amd", "autotune.json")
    best, _ = api.spline_plan_autotune(plan, bufs, reps=5, cache_path=cache)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    K = args.steps
    # points and results rotated over >= 2 GiB each, so that no step finds
    # them in the 256 MB last-level cache
    nrot = max(2, -(-(2 << 30) // (8 * M)))
    xq_h_t = torch.from_numpy(xq_h)
    rot = [{"xq": xq_h_t.cuda(), "yq": torch.empty(M, dtype=torch.float64, device="cuda"),
            "ypp": torch.empty(N, dtype=torch.float64, device="cuda")} for _ in range(nrot)]
    d1 = torch.empty(M, dtype=torch.float64, device="cuda")
    d2 = torch.empty_like(d1)
    it = [0]

    def build(r):
        api.spline_plan_run(plan, dict(bufs, ypp=r["ypp"]), stream=sp)

    def points(r, derivs=False):
        api.spline_batch_eval_points(bufs["koff"], qoff, bufs["x"], bufs["y"], r["ypp"], r["xq"], r["yq"],
                                     d1 if derivs else None, d2 if derivs else None, stream=sp)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(K):
            fn()
        e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) / K, (time.perf_counter() - t0) / K

    def rotated(fn):
        def step():
            fn(rot[it[0] % nrot])
            it[0] += 1
        return step

    build_ms, _ = timed(rotated(build))
    pts_ms, _ = timed(rotated(points))
    pts_d_ms, _ = timed(rotated(lambda r: points(r, True)))
    step_ms, step_s = timed(rotated(lambda r: (build(r), points(r))))
    # algorithmic bytes of the points launch: read the points and write the
    # values (16 per query), read x, y and y'' (24 per knot), and per curve
    # its two offsets (16); of the whole step, the build's 24 per knot more
    dbytes = 16.0 * M + 24.0 * N + 16.0 * b.count
    step_bytes = dbytes + 24.0 * N + 16.0 * b.count
    achieved = dbytes / (pts_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": (N + M) / step_s, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched_points: 4096 curves, sizes log-uniform 0.1x..10x of (13 knots, 2048 "
                               "points), explicit points U(x_0, x_{n-1}) per curve in random order; a build-only "
                               "plan then one spline_batch_eval_points launch (values), points and outputs rotated "
                               "over %.1f GB" % (nrot * 8 * M / 1e9),
                   "instances": b.count, "sum_n": N, "sum_m": M, "ends": "natural/flat/twist cycle", "seed": 0,
                   "points": "numpy default_rng(1)",
                   "build_tuning": {"block": best.block, "queries_per_tile": best.queries_per_tile,
                                    "grid_per_cu": best.grid_per_cu, "fused": best.fused}},
        "roofline": {"bound": "hbm", "kernel": "eval_points_batch", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("eval_points_batch", "batched_points"),
                     "algorithmic_bytes_per_launch": dbytes, "avg_launch_ms": pts_ms},
        "kernels_ms": {"build_only_plan": build_ms, "eval_points_batch_values": pts_ms,
                       "eval_points_batch_with_derivatives": pts_d_ms, "step_event_ms": step_ms},
        "step_frac": step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "with_derivatives": {"ms": pts_d_ms,
                             "frac": (dbytes + 16.0 * M) / (pts_d_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        import oracle
        # the oracle over the whole batch, curve by curve (y'' by banded
        # elimination, then every point bracketed and evaluated), single
        # thread, repeated for about --cpu-seconds
        reps = 0
        t0 = oracle.now()
        while True:
            for i in range(b.count):
                k0, k1, q0, q1 = b.koff[i], b.koff[i + 1], b.qoff[i], b.qoff[i + 1]
                o_ypp = oracle.second_derivatives(b.x[k0:k1], b.y[k0:k1], b.sd[i], b.ed[i])
                oracle.eval_points(b.x[k0:k1], b.y[k0:k1], o_ypp, xq_h[q0:q1])
            reps += 1
            if oracle.now() - t0 >= args.cpu_seconds:
                break
        t = oracle.now() - t0
        out["cpu_baseline"] = {"value": (N + M) * reps / t, "unit": UNIT, "cores": 1, "kind": "oracle",
                               "sample": "the whole batch (all %d curves: build and every point), %d repetitions "
                                         "in %.1f s, single thread" % (b.count, reps, t),
                               "ns_per_point": t / (M * reps) * 1e9}
    return out


def plain_context(args):
    """The single-curve configurations beside the batch: C2 (13,000 knots,
    2,048,000 queries) in one launch, and the same curve at m = 2^27 (out of
    the last-level cache), kernel time only."""
    import torch

    from paper_2001_09253_amd import api, workloads

    res = {}
    for name, n, m in (("plain", 13000, 2048000), ("plain2x", 13000, 1 << 27)):
        inst = workloads.single(0, n, m, bc=0)
        x = torch.from_numpy(inst.x).cuda()
        y = torch.from_numpy(inst.y).cuda()
        ypp = torch.empty_like(x)
        yq = torch.empty(m, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        sp = stream.cuda_stream
        reps = 200 if m < (1 << 24) else 20
        for _ in range(5):
            api.spline_solve_uniform(x, y, inst.start_deriv, inst.end_deriv, m, yq, ypp, stream=sp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            api.spline_solve_uniform(x, y, inst.start_deriv, inst.end_deriv, m, yq, ypp, stream=sp)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b_alg = 24.0 * n + 8.0 * m
        res[name] = {"n": n, "m": m, "ms": ms, "steps_per_s": (n + m) / (ms * 1e-3),
                     "frac": b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del x, y, ypp, yq
    return res


def bench_served(args):
    """Poisson arrivals through the request API: continuous batching against
    the plain one-request path, the same trace for both."""
    import numpy as np

    from paper_2001_09253_amd import api, serve, workloads

    dur = args.served_seconds + 1.0
    trace = workloads.poisson_trace(0, args.rate, dur, 0.1, 100.0)
    reqs = serve.make_requests(trace, 1)
    # one untimed pass through each path (library load, first launches)
    short = workloads.Trace(trace.t[:64] - trace.t[0], trace.n[:64], trace.m[:64])
    serve.replay(short, reqs[:64])
    serve.replay(short, reqs[:64], plain=True)
    res_b, _ = serve.replay(trace, reqs, warmup_s=1.0, budget=args.budget_gb << 30,
                            flags=0 if args.served_graph else api.NO_GRAPH)
    res_p, _ = serve.replay(trace, reqs, plain=True, warmup_s=1.0, budget=args.budget_gb << 30)
    sb, sp = res_b.summary(), res_p.summary()
    sel = trace.t >= 1.0
    nsum = int(trace.n[sel].sum())
    msum = int(trace.m[sel].sum())
    bytes_alg = 24.0 * nsum + 8.0 * msum
    gbs = bytes_alg / res_b.window_s / 1e9
    out = {
        "metric": METRIC, "value": sb["steps_per_s"], "unit": UNIT, "n_gpus": 1, "steps": res_b.requests,
        "warmup": int((~sel).sum()), "ms_per_step": sb["mean_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "served: Poisson %.0f req/s for %.0f s after 1 s warm-up, sizes log-uniform "
                               "0.1x..100x of (13, 2048), host result buffers" % (args.rate, args.served_seconds),
                   "requests": res_b.requests, "sum_n": nsum, "sum_m": msum,
                   "budget_bytes": args.budget_gb << 30, "graph": bool(args.served_graph)},
        "latency_ms": {"served_p50": sb["p50_ms"], "served_p99": sb["p99_ms"], "plain_p50": sp["p50_ms"],
                       "plain_p99": sp["p99_ms"], "served_max": sb["max_ms"], "plain_max": sp["max_ms"]},
        "served": sb, "plain": sp,
        "served_stats": res_b.stats,
        "roofline": {"bound": "hbm", "kernel": "served batches (offered load)", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": None, "avg_launch_ms": None},
    }
    # the paper's timing model (Gamma noise of mode Mo and sd sigma_inf +
    # sigma_0/n around a per-point baseline) fitted to the latency samples,
    # n = the request's knots + queries
    from paper_2001_09253_amd import timing_model
    tm = {}
    for name, res in (("served", res_b), ("plain", res_p)):
        try:
            tm[name] = timing_model.fit(res.sizes, res.latency_s)
        except Exception as e:  # a failed fit is reported, not fatal
            tm[name] = {"error": repr(e)}
    out["timing_model"] = tm
    # admission under a tight HBM budget (32 MB holds about 20 of the largest
    # requests), a shorter trace
    tr32 = workloads.poisson_trace(4, args.rate, 3.5, 0.1, 100.0)
    rq32 = serve.make_requests(tr32, 5)
    r32, _ = serve.replay(tr32, rq32, warmup_s=0.5, budget=32 << 20, flags=api.NO_GRAPH)
    out["budget_32mb"] = {"summary": r32.summary(), "stats": r32.stats}
    if args.sweep:
        rows = []
        for rate in (4000.0, 16000.0, 64000.0):
            tr = workloads.poisson_trace(2, rate, 2.0, 0.1, 100.0)
            rq = serve.make_requests(tr, 3)
            rb, _ = serve.replay(tr, rq, warmup_s=0.5, flags=api.NO_GRAPH)
            rp, _ = serve.replay(tr, rq, plain=True, warmup_s=0.5)
            rows.append({"rate": rate, "served": rb.summary(), "plain": rp.summary()})
        out["rate_sweep"] = rows
    if not args.no_cpu_baseline:
        import oracle
        # the oracle over the measured requests' inputs, OpenMP over
        # requests, for a bounded share of the trace
        idx = np.nonzero(sel)[0]
        t0 = oracle.now()
        done_steps = 0
        used = 1
        k = 0
        while oracle.now() - t0 < args.cpu_seconds and k < len(idx):
            chunk = idx[k:k + 256]
            koff = np.concatenate([[0], np.cumsum([reqs[r].n for r in chunk])]).astype(np.int64)
            qoff = np.concatenate([[0], np.cumsum([reqs[r].m for r in chunk])]).astype(np.int64)
            xs = np.concatenate([reqs[r].x for r in chunk])
            ys = np.concatenate([reqs[r].y for r in chunk])
            sds = np.array([reqs[r].sd for r in chunk])
            eds = np.array([reqs[r].ed for r in chunk])
            _, _, _, used = oracle.batch_uniform(koff, qoff, xs, ys, sds, eds)
            done_steps += int(koff[-1] + qoff[-1])
            k += len(chunk)
        t = oracle.now() - t0
        out["cpu_baseline"] = {"value": done_steps / t, "unit": UNIT, "cores": used, "kind": "oracle",
                               "sample": "first %d measured requests of the trace, back to back (no arrival "
                                         "gaps), OpenMP over requests, %.1f s" % (k, t)}
    return out


def served_context(seconds, rate=2000.0):
    """The served configuration, short: Poisson arrivals through the request
    API, continuous batching against the plain single-instance path (the
    same trace), latency from the scheduled arrival to the result."""
    from paper_2001_09253_amd import api, serve, workloads

    trace = workloads.poisson_trace(0, rate, seconds + 1.0, 0.1, 100.0)
    reqs = serve.make_requests(trace, 1)
    short = workloads.Trace(trace.t[:64] - trace.t[0], trace.n[:64], trace.m[:64])
    serve.replay(short, reqs[:64])
    serve.replay(short, reqs[:64], plain=True)
    res_b, _ = serve.replay(trace, reqs, warmup_s=1.0, flags=api.NO_GRAPH)
    res_p, _ = serve.replay(trace, reqs, plain=True, warmup_s=1.0)
    sb, sp = res_b.summary(), res_p.summary()
    return {"workload": "Poisson %.0f req/s for %.0f s after 1 s warm-up, sizes log-uniform 0.1x..100x of "
                        "(13, 2048), host result buffers, 200 GB budget" % (rate, seconds),
            "served_p50_ms": sb["p50_ms"], "served_p99_ms": sb["p99_ms"], "plain_p50_ms": sp["p50_ms"],
            "plain_p99_ms": sp["p99_ms"], "served_steps_per_s": sb["steps_per_s"],
            "plain_steps_per_s": sp["steps_per_s"], "requests": res_b.requests,
            "served_peak_device_bytes": res_b.stats.get("peak_device_bytes"),
            "served_peak_resident_bytes": res_b.stats.get("peak_resident_bytes")}


def bench_sweep(args):
    """The paper-style size sweep on one curve (m = n): sizes from its formula
    n = (r (sqrt(N) - sqrt(4)) + sqrt(4))^2 on a grid of r, N = 2^28, visited
    in shuffled order; the one-launch solve and the noop kernel (generate and
    bracket the queries only) per size, in ns per point.  Curves are prefixes
    of one seeded draw of the paper's generator (a prefix is itself a draw)."""
    import numpy as np
    import torch

    from paper_2001_09253_amd import api, workloads

    nmax = 1 << 28
    sizes = np.unique(workloads.sweep_sizes(7, 48, nmax=nmax, nmin=4))
    sizes = sizes[sizes >= 4]
    rng = np.random.default_rng(7)
    rng.shuffle(sizes)
    x, y = workloads.paper_curve(np.random.default_rng(0), nmax)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    del x, y
    ypp = torch.empty(nmax, dtype=torch.float64, device=dev)
    out = torch.empty(nmax, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    rows = []
    for n in sizes:
        n = int(n)
        m = n
        xs, ys = xd[:n], yd[:n]

        def solve():
            api.spline_solve_uniform(xs, ys, 1e32, 1e32, m, out[:m], ypp[:n])

        def noop():
            api.spline_noop_uniform(xs, m, out[:m])
        st = torch.zeros((1,), dtype=torch.int32, device=dev)
        api.spline_solve_uniform(xs, ys, 1e32, 1e32, m, out[:m], ypp[:n], st)
        if int(st.cpu()[0]) != api.OK:
            raise RuntimeError("sweep curve of %d knots rejected (status %d)" % (n, int(st.cpu()[0])))
        res = {}
        for name, fn in (("solve", solve), ("noop", noop)):
            fn()
            torch.cuda.synchronize()
            reps = int(min(200, max(3, 2e8 // (n + 1))))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name] = e0.elapsed_time(e1) / reps
        b_alg = 24.0 * n + 8.0 * m
        rows.append({"n": n, "m": m, "solve_us": res["solve"] * 1e3, "noop_us": res["noop"] * 1e3,
                     "solve_ns_per_point": res["solve"] * 1e6 / m, "noop_ns_per_point": res["noop"] * 1e6 / m,
                     "solve_gbs": b_alg / (res["solve"] * 1e-3) / 1e9})
    rows.sort(key=lambda r: r["n"])
    big = rows[-1]
    out_d = {
        "metric": METRIC, "value": (big["n"] + big["m"]) / (big["solve_us"] * 1e-6), "unit": UNIT, "n_gpus": 1,
        "steps": len(rows), "warmup": 1, "ms_per_step": big["solve_us"] * 1e-3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sweep: 1 curve per size, m = n, %d sizes from 4 to 2^28 (the paper's size formula), "
                               "shuffled" % len(rows), "seed": 0},
        "roofline": {"bound": "hbm", "kernel": "solve_uniform", "achieved": big["solve_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": big["solve_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": 24.0 * big["n"] + 8.0 * big["m"],
                     "avg_launch_ms": big["solve_us"] * 1e-3},
        "sweep": rows,
    }
    if not args.no_cpu_baseline:
        import oracle
        # the oracle single-threaded, as in the paper, at the sweep's sizes up
        # to 2^20 (bounded by --cpu-seconds overall)
        xh, yh = workloads.paper_curve(np.random.default_rng(0), 1 << 20)
        cpu = []
        t_all = oracle.now()
        for r in rows:
            n = r["n"]
            if n > (1 << 20) or oracle.now() - t_all > args.cpu_seconds:
                continue
            reps = 0
            t0 = oracle.now()
            while True:
                oracle.spline_uniform(xh[:n], yh[:n], 1e32, 1e32, n)
                reps += 1
                if oracle.now() - t0 > 0.05:
                    break
            cpu.append({"n": n, "ns_per_point": (oracle.now() - t0) / reps / n * 1e9})
        out_d["cpu_baseline"] = {"value": None, "unit": "ns/point", "cores": 1, "kind": "oracle",
                                 "sample": "single thread, m = n, sizes of the sweep up to 2^20", "points": cpu}
    return out_d


def bench_copy(args):
    """Calibration only: a plain device-to-device copy of 256 MiB (reads and
    writes 256 MiB per launch), the reference the HBM traffic counters of the
    other workloads are scaled by."""
    import torch

    nbytes = 256 << 20
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    return {"metric": "copy calibration (not a product metric)", "value": 2.0 * nbytes / (ms * 1e-3) / 1e9,
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy: 256 MiB device to device", "bytes_read": nbytes, "bytes_written": nbytes}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batched",
                    choices=["plain", "small", "plain2x", "points", "batched_points", "long", "batched", "mixed",
                             "served", "copy", "sweep"])
    ap.add_argument("--sorted", action="store_true", help="points: sorted query points")
    ap.add_argument("--variant", default=None,
                    choices=["newint", "newint__orig", "newint__noinv", "splint_one__div", "splint_one__mul", "horner"],
                    help="single-curve workloads: time this evaluation formula on the one-launch kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--rate", type=float, default=2000.0, help="served: arrivals per second")
    ap.add_argument("--served-seconds", type=float, default=10.0, help="served: measured seconds")
    ap.add_argument("--budget-gb", type=int, default=200, help="served: HBM admission budget")
    ap.add_argument("--served-graph", action="store_true", help="served: capture each batch as a hipGraph")
    ap.add_argument("--sweep", action="store_true", help="served: also a short sweep of arrival rates")
    ap.add_argument("--no-context", action="store_true",
                    help="batched: skip the single-curve and served context measurements")
    ap.add_argument("--context-seconds", type=float, default=4.0,
                    help="batched: measured seconds of each served path in the context")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the spline path runs on one MI355X, and how it "
              "would shard is a design note, not a code path (--gpus %d is not supported)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "plain":
        out = bench_single(args, 13000, 2048000, "plain: 1 curve, n=13000, m=2048000 uniform queries")
    elif args.workload == "small":
        out = bench_single(args, 13, 2048, "small: 1 curve, n=13, m=2048 uniform queries")
    elif args.workload == "plain2x":
        out = bench_single(args, 13000, 1 << 27, "plain2x: 1 curve, n=13000, m=2^27 uniform queries")
    elif args.workload == "points":
        out = bench_points(args, args.sorted)
    elif args.workload == "batched_points":
        out = bench_batched_points(args)
    elif args.workload == "long":
        out = bench_single(args, 1 << 28, 1 << 28, "long: 1 curve, n=m=2^28 (the size sweep's largest point)",
                           cpu_sample=1 << 22)
    elif args.workload in ("batched", "mixed"):
        from paper_2001_09253_amd import api
        out = bench_batched(args, api.FP64 if args.workload == "batched" else api.FP32_REFINE)
        if args.workload == "batched" and not args.no_context:
            # beside the batch: the single-curve kernel on C2 and C2x, and the
            # served form against the plain single-instance path
            out["context"] = {"single_curve": plain_context(args),
                              "served": served_context(args.context_seconds)}
    elif args.workload == "copy":
        out = bench_copy(args)
    elif args.workload == "sweep":
        out = bench_sweep(args)
    else:
        out = bench_served(args)
    if "roofline" in out and out["roofline"].get("achieved") and args.workload != "copy":
        add_copy_ceiling(out)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
