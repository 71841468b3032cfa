"""rocprofv3 output summaries: per-kernel trace statistics, per-dispatch
counter means, and counter-derived HBM traffic of one kernel.

    python -m paper_1908_06094_amd.profsum trace DIR
    python -m paper_1908_06094_amd.profsum counters DIR
    python -m paper_1908_06094_amd.profsum traffic --fetch DIR --write DIR --kernel SUBSTR \
        --copy-bytes N [--kind KIND --out JSON --workload TEXT --command CMD ...]

``traffic`` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
kernels whose name contains SUBSTR by the ratio each counter shows for a plain
device copy of N bytes in the same run, and records the hash of the kernel
sources so that a reader can tell whether the record still describes them.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sqlite3
import sys

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# the sources the fused corrective-pass kernel is compiled from
PASS_KERNEL_SOURCES = ("fused.hpp", "common.hpp")


def kernel_source_sha(names=PASS_KERNEL_SOURCES):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def from_db(path):
    con = sqlite3.connect(path)
    q = ("select s.kernel_name, count(*), avg(d.end - d.start), sum(d.end - d.start), min(d.end - d.start), "
         "max(d.end - d.start) from rocpd_kernel_dispatch d join rocpd_info_kernel_symbol s "
         "on d.kernel_id = s.id group by s.kernel_name order by sum(d.end - d.start) desc")
    return [(r[0], r[1], r[2] / 1e3, r[3] / 1e3, r[4] / 1e3, r[5] / 1e3) for r in con.execute(q)]


def from_csv(path):
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e3,
                        float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    return out


def summarise(path):
    """[(kernel, calls, avg_us, total_us, min_us, max_us)] of a kernel trace."""
    if os.path.isdir(path):
        hits = glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)
        if hits:
            return from_csv(hits[0])
        hits = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
        return from_db(hits[0])
    return from_csv(path) if path.endswith(".csv") else from_db(path)


def last_launches_mean(path, kernel_substr, n):
    """Mean duration (us) of the last `n` dispatches of the kernel whose name
    contains `kernel_substr`, from a rocprofv3 per-dispatch kernel trace CSV
    directory: the timed launches of a run whose first ones are warm-up."""
    hits = glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)
    spans = []
    with open(hits[0]) as f:
        for r in csv.DictReader(f):
            if kernel_substr in r["Kernel_Name"]:
                spans.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    spans.sort()
    last = spans[-n:]
    return sum(e - s for s, e in last) / len(last) / 1e3


def counters(path):
    """{kernel name: {counter: mean value per dispatch}} from a rocprofv3 counter CSV directory."""
    hits = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(hits[0]) as f:
        for r in csv.DictReader(f):
            agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}


def traffic(fetch_dir, write_dir, kernel_substr, copy_bytes):
    """HBM bytes per launch (mean over the matching kernels) from the two counter runs."""
    f, w = counters(fetch_dir), counters(write_dir)
    copy_f = next(v["FETCH_SIZE"] for k, v in f.items() if "copyBuffer" in k)
    copy_w = next(v["WRITE_SIZE"] for k, v in w.items() if "copyBuffer" in k)
    ff = copy_bytes / 1024.0 / copy_f
    wf = copy_bytes / 1024.0 / copy_w
    names = sorted(k for k in f if kernel_substr in k)
    if not names:
        raise SystemExit(f"no kernel matching {kernel_substr!r} in {fetch_dir}")
    per = {k: (f[k]["FETCH_SIZE"] * ff + w[k]["WRITE_SIZE"] * wf) * 1024.0 for k in names}
    return {"copy_calibration": {"copy_bytes": copy_bytes, "fetch_factor": round(ff, 5), "write_factor": round(wf, 5)},
            "fetch_kib_per_dispatch": {k: f[k]["FETCH_SIZE"] for k in names},
            "write_kib_per_dispatch": {k: w[k]["WRITE_SIZE"] for k in names},
            "bytes_per_launch": int(round(sum(per.values()) / len(per)))}


def _main(argv):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("path")
    c = sub.add_parser("counters")
    c.add_argument("path")
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--kind", default="pass", help="the timing kind bench.py reports the kernel under")
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--workload", default="")
    r.add_argument("--command", action="append", default=[])
    r.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(f"{'kernel':<70} {'calls':>6} {'avg_us':>10} {'total_us':>11} {'min_us':>9} {'max_us':>9}")
        for name, n, avg, tot, mn, mx in summarise(a.path):
            print(f"{name[:70]:<70} {n:>6} {avg:>10.1f} {tot:>11.1f} {mn:>9.1f} {mx:>9.1f}")
    elif a.cmd == "counters":
        for k, d in sorted(counters(a.path).items()):
            print(k[:70], " ".join(f"{n}={v:.0f}" for n, v in sorted(d.items())))
    else:
        rec = {"kernel": a.kernel, "kernel_kind": a.kind, "workload": a.workload, "source_sha256": kernel_source_sha(),
               "commands": a.command}
        rec.update(traffic(a.fetch, a.write, a.kernel, a.copy_bytes))
        text = json.dumps(rec, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)


if __name__ == "__main__":
    _main(sys.argv[1:])
