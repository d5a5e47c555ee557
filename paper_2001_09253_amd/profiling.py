"""Summaries of rocprofv3 output for the committed measurement record.

    python -m paper_2001_09253_amd.profiling stats <rocprofv3 dir> <out.txt> <command...>
        writes the per-kernel duration table of a --kernel-trace --stats run
        (average, and the median dispatch from the trace), headed by the
        command that produced it and $PROFILE_NOTE, if set; with
        $PROFILE_LAST = K also each kernel's last K dispatches (a bench
        run's timed launches);
    python -m paper_2001_09253_amd.profiling traffic <kernel> <workload> <fetch dir> <write dir>
        <copy fetch dir> <copy write dir> <copy bytes> [<kernel substring>]
        scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over the
        dispatches of the kernel) by what the same counters read for a plain
        copy of known size, and records the bytes per launch in
        profiles/pmc_traffic.json under "<kernel>|<workload>" together with a
        hash of the kernel sources (a reading taken on other sources is not
        reported by bench.py).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_09253_amd", "csrc")
TRAFFIC = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _one(pattern):
    hits = glob.glob(pattern, recursive=True)
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _kernel_rows(prof_dir):
    """Per-kernel calls and durations (ns) from a --stats CSV, or, without
    one, from the run's rocpd database."""
    hits = glob.glob(os.path.join(prof_dir, "**", "*kernel_stats.csv"), recursive=True)
    if hits:
        with open(hits[0]) as f:
            return list(csv.DictReader(f))
    import sqlite3
    con = sqlite3.connect(_one(os.path.join(prof_dir, "**", "*.db")))
    q = ("select name, count(*), avg(duration), min(duration), max(duration) from kernels "
         "group by name order by sum(duration) desc")
    return [{"Name": r[0], "Calls": str(r[1]), "AverageNs": r[2], "MinNs": r[3], "MaxNs": r[4]}
            for r in con.execute(q)]


def _median(v):
    v = sorted(v)
    return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])


def _durations(prof_dir):
    """Dispatch durations (ns) per kernel in dispatch order, from the run's
    kernel trace (empty without one)."""
    hits = glob.glob(os.path.join(prof_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not hits:
        return {}
    rows = []
    with open(hits[0]) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), r["Kernel_Name"],
                         int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    per = {}
    for _, name, d in rows:
        per.setdefault(name, []).append(d)
    return per


def _medians(prof_dir):
    """Median dispatch duration (ns) per kernel from the run's kernel trace,
    if the trace is there."""
    return {k: _median(v) for k, v in _durations(prof_dir).items()}


def stats(prof_dir, out_path, command, note=None, last=0):
    """The summary; with last > 0 also the average and median of each
    kernel's last `last` dispatches (the timed launches of a bench run, which
    come after its warm-up and context launches)."""
    rows = _kernel_rows(prof_dir)
    med = _medians(prof_dir)
    durs = _durations(prof_dir) if last > 0 else {}
    lines = ["# rocprofv3 --kernel-trace --stats", "# command: " + command,
             "# kernel sources: " + kernel_source_hash()]
    if note:
        lines += ["# " + line for line in note.splitlines()]
    lines += ["", "%-72s %7s %12s %12s %12s %12s" % ("kernel", "calls", "avg_us", "median_us", "min_us", "max_us")]
    for r in rows:
        name = r["Name"] if len(r["Name"]) <= 72 else r["Name"][:69] + "..."
        m = med.get(r["Name"])
        lines.append("%-72s %7s %12.3f %12s %12.3f %12.3f" % (name, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                           "%.3f" % (m / 1e3) if m is not None else "-",
                                                           float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    if last > 0 and durs:
        lines += ["", "last %d dispatches of each kernel (the timed launches):" % last,
                  "%-72s %7s %12s %12s" % ("kernel", "calls", "avg_us", "median_us")]
        for r in rows:
            v = durs.get(r["Name"], [])[-last:]
            if not v:
                continue
            name = r["Name"] if len(r["Name"]) <= 72 else r["Name"][:69] + "..."
            lines.append("%-72s %7d %12.3f %12.3f" % (name, len(v), sum(v) / len(v) / 1e3, _median(v) / 1e3))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(prof_dir, counter, substr):
    path = _one(os.path.join(prof_dir, "**", "*counter_collection.csv"))
    vals = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and substr in r["Kernel_Name"]:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError("no %s for %s in %s" % (counter, substr, path))
    return sum(vals) / len(vals), len(vals)


def traffic(kernel, workload, fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, substr=None):
    substr = substr or kernel
    fk, nf = _counter(fetch_dir, "FETCH_SIZE", substr)
    wk, nw = _counter(write_dir, "WRITE_SIZE", substr)
    cf, _ = _counter(cfetch_dir, "FETCH_SIZE", "copy")
    cw, _ = _counter(cwrite_dir, "WRITE_SIZE", "copy")
    copy_bytes = float(copy_bytes)
    fscale = copy_bytes / (cf * 1024.0)   # bytes per KiB the counter reports
    wscale = copy_bytes / (cw * 1024.0)
    read_b = fk * 1024.0 * fscale
    write_b = wk * 1024.0 * wscale
    rec = {"bytes_per_launch": read_b + write_b, "read_bytes": read_b, "write_bytes": write_b,
           "fetch_kib": fk, "write_kib": wk, "dispatches": [nf, nw],
           "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes": copy_bytes,
           "scale_fetch": fscale, "scale_write": wscale, "source_hash": kernel_source_hash()}
    data = {}
    if os.path.exists(TRAFFIC):
        with open(TRAFFIC) as f:
            data = json.load(f)
    data["%s|%s" % (kernel, workload)] = rec
    os.makedirs(os.path.dirname(TRAFFIC), exist_ok=True)
    with open(TRAFFIC, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(rec))


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]), os.environ.get("PROFILE_NOTE"),
              int(os.environ.get("PROFILE_LAST", "0")))
    elif len(sys.argv) >= 9 and sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    else:
        print(__doc__)
        sys.exit(2)
