"""Summarise rocprofv3 CSV output of bench.py runs into short text tables.

  python -m paper_2509_03024_amd.profsummary trace <prefix>_kernel_trace.csv [KERNEL=N ... | bench.json]
  python -m paper_2509_03024_amd.profsummary hbm <fetch_counter_collection.csv> <write_counter_collection.csv> [KERNEL=N ... | bench.json]

trace: per kernel dispatches, total and average duration; for each KERNEL=N
       the average over its last N dispatches (N = the launch count bench.py
       reports for the timed steps, which end the run).  Given the JSON line
       bench.py printed instead, N comes from its per-kernel table and the
       summary sets the HIP-event average beside the profiler's.
counters: every counter of a --pmc run, mean per dispatch over each kernel's
       last N dispatches.
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
    m = re.search(r"k_ntt_pass<\d+, (true|false), (true|false)(?:, (?:true|false))?>", name)
    if m:
        return "k_ntt_pass<%s,%s>" % ("cols" if m.group(1) == "true" else "rows",
                                      "inv" if m.group(2) == "true" else "fwd")
    m = re.search(r"(k_[a-z_]+)", name)
    return m.group(1) if m else name[:60]


def _lastn(argv):
    """KERNEL=N arguments, or one bench.py JSON file: {kernel: (N, HIP-event average in us or None)}."""
    out = {}
    for a in argv:
        if a.endswith(".json"):
            import json
            line = [x for x in open(a).read().splitlines() if x.startswith("{")][-1]
            for k, v in json.loads(line)["kernels"].items():
                out[k] = (int(v["launches"]), float(v["avg_us"]))
            continue
        k, v = a.rsplit("=", 1)
        out[k] = (int(v), None)
    return out


def _steps(argv):
    """Timed steps of the bench.py JSON line among the arguments, or None."""
    for a in argv:
        if a.endswith(".json"):
            import json
            line = [x for x in open(a).read().splitlines() if x.startswith("{")][-1]
            return int(json.loads(line).get("steps", 0)) or None
    return None


def trace(path, last):
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows = sorted(((sum(d for _, d in v), k, len(v)) for k, v in per.items()), reverse=True)
    print(f"{'kernel':30s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s}")
    for tot, k, n in rows:
        print(f"{k:30s} {n:7d} {tot / 1e6:10.3f} {tot / n / 1e3:10.2f}")
    for k, (n, ev) in last.items():
        v = sorted(per.get(k, []))[-n:]
        if v:
            avg = sum(d for _, d in v) / len(v) / 1e3
            cmp = f" (HIP events in bench.py: {ev:.2f} us, ratio {avg / ev:.3f})" if ev else ""
            print(f"timed steps: {k} average over its last {len(v)} dispatches = {avg:.2f} us{cmp}")


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


def hbm(fetch_path, write_path, last, steps=None):
    f, fc = _counters(fetch_path, "FETCH_SIZE")
    w, wc = _counters(write_path, "WRITE_SIZE")
    sf, sw = CALIB_KIB / fc, CALIB_KIB / wc
    print(f"calibration copy (512 MiB): FETCH_SIZE {fc:.1f} KiB -> scale {sf:.3f}; "
          f"WRITE_SIZE {wc:.1f} KiB -> scale {sw:.3f}")
    total = 0.0
    for k, (n, _) in last.items():
        fv = [v for _, v in sorted(f.get(k, []))[-n:]]
        wv = [v for _, v in sorted(w.get(k, []))[-n:]]
        if fv and wv:
            fb = sum(fv) / len(fv) * sf * 1024
            wb = sum(wv) / len(wv) * sw * 1024
            total += (fb + wb) * n
            print(f"timed steps: {k} over its last {len(fv)} dispatches: fetch {fb / 1e6:.1f} MB, "
                  f"write {wb / 1e6:.1f} MB, traffic {(fb + wb) / 1e6:.1f} MB per launch")
    if steps:
        print(f"timed steps: all listed kernels, traffic {total / steps / 1e9:.1f} GB per step ({steps} steps)")


def counters(path, last):
    per = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])][r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    for k, (n, _) in last.items():
        if k not in per:
            continue
        vals = []
        for cname in sorted(per[k]):
            v = [x for _, x in sorted(per[k][cname])[-n:]]
            vals.append(f"{cname}={sum(v) / len(v):.4g}")
        print(f"timed steps: {k} (last {n} dispatches, mean per dispatch): " + " ".join(vals))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], _lastn(sys.argv[3:]))
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], _lastn(sys.argv[3:]))
    else:
        hbm(sys.argv[2], sys.argv[3], _lastn(sys.argv[4:]), _steps(sys.argv[4:]))
