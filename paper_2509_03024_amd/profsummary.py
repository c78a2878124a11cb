"""Summarise rocprofv3 CSV output of bench.py runs into short text tables.

  python -m paper_2509_03024_amd.profsummary trace <prefix>_kernel_trace.csv [KERNEL=N ...]
  python -m paper_2509_03024_amd.profsummary hbm <fetch_counter_collection.csv> <write_counter_collection.csv> [KERNEL=N ...]

trace: per kernel dispatches, total and average duration; for each KERNEL=N
       the average over its last N dispatches (N = the launch count bench.py
       reports for the timed step, which ends the run).
hbm:   FETCH_SIZE / WRITE_SIZE per dispatch (KiB), scaled by the reading of the
       512 MiB calibration copy (bench.py --calib-copy): the copy must move
       524,288 KiB each way.  For each KERNEL=N the mean over its last N
       dispatches, in bytes per launch.
"""
import csv
import re
import sys
from collections import defaultdict

CALIB_KIB = 524288.0


def short(name):
    """Kernel name as bench.py's per-kernel profile reports it."""
    m = re.search(r"k_ntt_pass<\d+, (true|false), (true|false)>", name)
    if m:
        return "k_ntt_pass<%s,%s>" % ("cols" if m.group(1) == "true" else "rows",
                                      "inv" if m.group(2) == "true" else "fwd")
    m = re.search(r"(k_[a-z_]+)", name)
    return m.group(1) if m else name[:60]


def _lastn(argv):
    out = {}
    for a in argv:
        k, v = a.rsplit("=", 1)
        out[k] = int(v)
    return out


def trace(path, last):
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows = sorted(((sum(d for _, d in v), k, len(v)) for k, v in per.items()), reverse=True)
    print(f"{'kernel':30s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s}")
    for tot, k, n in rows:
        print(f"{k:30s} {n:7d} {tot / 1e6:10.3f} {tot / n / 1e3:10.2f}")
    for k, n in last.items():
        v = sorted(per.get(k, []))[-n:]
        if v:
            print(f"timed step: {k} average over its last {len(v)} dispatches = "
                  f"{sum(d for _, d in v) / len(v) / 1e3:.2f} us")


def _counters(path, cname):
    per = defaultdict(list)
    calib = None
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != cname:
            continue
        v = float(r["Counter_Value"])
        per[short(r["Kernel_Name"])].append((int(r["Dispatch_Id"]), v))
        if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 131072:
            calib = v
    return per, calib


def hbm(fetch_path, write_path, last):
    f, fc = _counters(fetch_path, "FETCH_SIZE")
    w, wc = _counters(write_path, "WRITE_SIZE")
    sf, sw = CALIB_KIB / fc, CALIB_KIB / wc
    print(f"calibration copy (512 MiB): FETCH_SIZE {fc:.1f} KiB -> scale {sf:.3f}; "
          f"WRITE_SIZE {wc:.1f} KiB -> scale {sw:.3f}")
    for k, n in last.items():
        fv = [v for _, v in sorted(f.get(k, []))[-n:]]
        wv = [v for _, v in sorted(w.get(k, []))[-n:]]
        if fv and wv:
            fb = sum(fv) / len(fv) * sf * 1024
            wb = sum(wv) / len(wv) * sw * 1024
            print(f"timed step: {k} over its last {len(fv)} dispatches: fetch {fb / 1e6:.1f} MB, "
                  f"write {wb / 1e6:.1f} MB, traffic {(fb + wb) / 1e6:.1f} MB per launch")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], _lastn(sys.argv[3:]))
    else:
        hbm(sys.argv[2], sys.argv[3], _lastn(sys.argv[4:]))
