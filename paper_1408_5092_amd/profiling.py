"""Summaries of rocprofv3 CSV output for the benchmark's timed region.

The library launches an empty kernel, k_profile_mark, whenever its kernel
timing is switched on or off; bench.py switches it on for exactly the timed
steps, so the dispatches between the first and the last k_profile_mark are
the timed region.

  python -m paper_1408_5092_amd.profiling trace DIR [--delete-csv]
      per-kernel calls / total / average duration in the window, from
      DIR/*_kernel_trace.csv (rocprofv3 --kernel-trace --output-format csv)
  python -m paper_1408_5092_amd.profiling counters DIR [--delete-csv]
      per-kernel average counter value (KiB) per dispatch in the window and
      the value of the largest plain copy (bench.py --copy-calibration),
      from DIR/*_counter_collection.csv (rocprofv3 --pmc COUNTER)
  python -m paper_1408_5092_amd.profiling traffic FETCH_DIR WRITE_DIR KERNEL[,KERNEL...] COPY_BYTES
      HBM bytes per dispatch of KERNEL (several names: their dispatches
      together): each counter scaled by the ratio of
      the copy's true bytes (COPY_BYTES read, COPY_BYTES written) to what
      that counter reported for the copy

Each command writes a JSON summary next to the CSV files and prints it.
"""
import collections
import csv
import glob
import json
import os
import re
import sys


def _short(name):
    m = re.search(r"(k_\w+(<[\w, ]+>)?|__amd_\w+)", name)
    return m.group(1) if m else name[:60]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, f"*{suffix}"))
    if not files:
        raise FileNotFoundError(f"no *{suffix} in {d}")
    return files[0]


def trace(d, delete=False):
    path = _csv(d, "_kernel_trace.csv")
    with open(path) as f:
        disp = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in csv.DictReader(f))
    marks = [s for s, _, n in disp if "k_profile_mark" in n]
    t0, t1 = (marks[0], marks[-1]) if len(marks) >= 2 else (disp[0][0], disp[-1][1])
    agg = collections.defaultdict(list)
    for s, e, n in disp:
        if t0 < s < t1:
            agg[_short(n)].append((e - s) * 1e-3)
    out = {"window_ms": (t1 - t0) * 1e-6,
           "kernels": {n: {"calls": len(v), "total_ms": sum(v) / 1e3, "avg_us": sum(v) / len(v),
                           "min_us": min(v), "max_us": max(v)} for n, v in agg.items()}}
    with open(os.path.join(d, "window_summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    if delete:
        os.remove(path)
    return out


def counters(d, delete=False):
    path = _csv(d, "_counter_collection.csv")
    with open(path) as f:
        rows = list(csv.DictReader(f))
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: int(r[key]))
    marks = [i for i, r in enumerate(rows) if "k_profile_mark" in r["Kernel_Name"]]
    lo, hi = (marks[0], marks[-1]) if len(marks) >= 2 else (-1, len(rows))
    win = collections.defaultdict(list)
    copy = None
    for i, r in enumerate(rows):
        v = float(r["Counter_Value"])
        if "copyBuffer" in r["Kernel_Name"]:
            g = int(r.get("Grid_Size") or 0)
            if copy is None or g > copy[0]:
                copy = (g, v)
        if lo < i < hi:
            win[_short(r["Kernel_Name"])].append(v)
    out = {"counter": rows[0].get("Counter_Name"), "copy_kib": copy[1] if copy else None,
           "kernels": {n: {"dispatches": len(v), "avg_kib": sum(v) / len(v)} for n, v in win.items()}}
    with open(os.path.join(d, "counter_summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    if delete:
        os.remove(path)
    return out


def traffic(fetch_dir, write_dir, kernel, copy_bytes):
    """KERNEL may list several comma-separated names (launch shapes of one kernel
    kind); their per-dispatch averages are combined weighted by dispatches."""
    fs = json.load(open(os.path.join(fetch_dir, "counter_summary.json")))
    ws = json.load(open(os.path.join(write_dir, "counter_summary.json")))
    kib = copy_bytes / 1024.0
    f_scale, w_scale = kib / fs["copy_kib"], kib / ws["copy_kib"]
    names = kernel.split(",")

    def avg(summary):
        rows = [summary["kernels"][n] for n in names if n in summary["kernels"]]
        n = sum(r["dispatches"] for r in rows)
        return sum(r["avg_kib"] * r["dispatches"] for r in rows) / n if n else 0.0, n

    (fk, nf), (wk, _) = avg(fs), avg(ws)
    return {"kernel": kernel, "dispatches": nf, "fetch_kib": fk, "write_kib": wk, "fetch_scale": f_scale,
            "write_scale": w_scale, "bytes_per_dispatch": 1024.0 * (fk * f_scale + wk * w_scale)}


def main(argv):
    if len(argv) >= 2 and argv[0] in ("trace", "counters"):
        fn = trace if argv[0] == "trace" else counters
        print(json.dumps(fn(argv[1], "--delete-csv" in argv), indent=1))
    elif len(argv) == 5 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], float(argv[4])), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
