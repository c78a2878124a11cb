"""Summarise a rocprofv3 kernel trace (CSV) of bench.py into a short text table.

Usage: python -m paper_2509_03024_amd.profsummary <prefix>_kernel_trace.csv [--last-step-launches K=N ...]

Prints per kernel: dispatches, total and average duration.  Because the
trace also covers set-up work (key generation, imports), the average of a
kernel over the benchmark's timed step is taken from its last N dispatches,
where N is the launch count bench.py reports for that kernel.
"""
import csv
import re
import sys
from collections import defaultdict


def short(name):
    """Kernel name as bench.py's per-kernel profile reports it."""
    m = re.search(r"k_ntt_pass<\d+, (true|false), (true|false)>", name)
    if m:
        return "k_ntt_pass<%s,%s>" % ("cols" if m.group(1) == "true" else "rows",
                                      "inv" if m.group(2) == "true" else "fwd")
    m = re.search(r"(k_[a-z_]+)", name)
    return m.group(1) if m else name[:60]


def main(argv):
    path = argv[0]
    last = {}
    for a in argv[1:]:
        if "=" in a:
            k, v = a.split("=", 1)
            last[k] = int(v)
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per[short(r["Kernel_Name"])].append((int(r["Start_Timestamp"]), d))
    rows = []
    for k, v in per.items():
        v.sort()
        tot = sum(d for _, d in v)
        rows.append((tot, k, len(v), tot / len(v)))
    rows.sort(reverse=True)
    print(f"{'kernel':42s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s}")
    for tot, k, n, avg in rows:
        print(f"{k:42s} {n:7d} {tot / 1e6:10.3f} {avg / 1e3:10.2f}")
    for k, n in last.items():
        v = sorted(per.get(k, []))[-n:]
        if v:
            print(f"timed-step average of {k} over its last {len(v)} dispatches: "
                  f"{sum(d for _, d in v) / len(v) / 1e3:.2f} us")


if __name__ == "__main__":
    main(sys.argv[1:])
