"""Summarise a rocprofv3 kernel trace (rocpd SQLite or kernel_stats CSV) per kernel."""
from __future__ import annotations

import csv
import glob
import os
import sqlite3
import sys


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
    if os.path.isdir(path):
        hits = glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)
        if hits:
            return from_csv(hits[0])
        hits = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
        return from_db(hits[0])
    return from_csv(path) if path.endswith(".csv") else from_db(path)


if __name__ == "__main__":
    rows = summarise(sys.argv[1])
    print(f"{'kernel':<70} {'calls':>6} {'avg_us':>10} {'total_us':>11} {'min_us':>9} {'max_us':>9}")
    for name, n, avg, tot, mn, mx in rows:
        print(f"{name[:70]:<70} {n:>6} {avg:>10.1f} {tot:>11.1f} {mn:>9.1f} {mx:>9.1f}")
