"""Summaries of rocprofv3 output for the sweep kernels.

  python profile_summary.py stats <dir> <out.txt> <command...>
      per-kernel table (calls, average and total duration) from the
      *_kernel_stats.csv of a `rocprofv3 --kernel-trace --stats --output-format csv` run
  python profile_summary.py traffic <key> <kernel-substring> <fetch_dir> <write_dir>
      <copy_fetch_dir> <copy_write_dir> <copy_bytes> <out.txt> <traffic.json>
      HBM bytes per dispatch of one kernel from FETCH_SIZE and WRITE_SIZE runs (KiB per
      dispatch), each scaled so that a plain copy of copy_bytes reads as copy_bytes; the entry
      of traffic.json records a sha256 of the sweep kernels' source and build flags
      (kernel_source_sha) the counters were taken on.
  python profile_summary.py traffic_per_call <calls> <key> ... (as traffic)
      the same for kernels launched several times per call: the counters of all
      dispatches summed and divided by the number of calls.
  python profile_summary.py spans <dir> <kernel-substring> <launches-per-call> <out.txt>
      appends to out.txt, from the *_kernel_trace.csv of the same run, the time from the
      first start to the last end of each call's launches of one kernel (the launches of a
      call may run on several streams at once), their summed durations and the queues used.
  python profile_summary.py counters <kernel-substring> <out.txt> <dir>[,<dir>...] <command...>
      every counter of the `rocprofv3 --pmc` runs in the listed directories for one
      kernel, averaged per dispatch.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2001_09196_amd")


def _one(pattern):
    fs = sorted(glob.glob(pattern, recursive=True))
    if not fs:
        raise SystemExit(f"no file matches {pattern}")
    return fs[0]


def stats(d, out, command):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':70s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:25]:
        name = r["Name"]
        if len(name) > 70:
            name = name[:67] + "..."
        lines.append(f"{name:70s} {int(r['Calls']):7d} {float(r['AverageNs'])/1e3:10.2f} "
                     f"{float(r['TotalDurationNs'])/1e6:10.3f} {float(r['Percentage']):6.2f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(d, counter, kernel, per_call=0):
    """Median over dispatches (KiB), or, with per_call = k > 0, the sum over all
    dispatches divided by k (kernels launched k times per call)."""
    vals = {}
    for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
        if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
            vals.setdefault(r["Dispatch_Id"], 0.0)
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel} in {d}")
    if per_call > 0:
        return sum(vals.values()) / per_call, len(vals)
    v = sorted(vals.values())
    return v[len(v) // 2], len(v)   # median over dispatches, KiB


SWEEP_SOURCES = ("csrc/sweep.hip", "csrc/sn_device.hpp", "csrc/sn_kernels.hpp", "build.py")
HP_SOURCES = ("csrc/hp.hip", "csrc/hp.hpp", "csrc/sn_device.hpp", "csrc/sn_kernels.hpp", "build.py")


def sources_of(kernel: str):
    """The files that decide a kernel's code: the order-p kernels' (hp.hip)
    or the Q1 sweep kernels' (sweep.hip), with the headers and build flags."""
    return HP_SOURCES if "_hp" in kernel else SWEEP_SOURCES


def kernel_source_sha(files=SWEEP_SOURCES) -> str:
    """sha256 over the files that decide the sweep kernels' code: their
    source, the device header, the launch header and the build flags."""
    h = hashlib.sha256()
    for rel in files:
        h.update(open(os.path.join(HERE, rel), "rb").read())
    return h.hexdigest()


def traffic(key, kernel, fdir, wdir, cfdir, cwdir, copy_bytes, out, jpath, command, per_call=0):
    copy_bytes = float(copy_bytes)
    cf, _ = _per_dispatch(cfdir, "FETCH_SIZE", "copy")
    cw, _ = _per_dispatch(cwdir, "WRITE_SIZE", "copy")
    sf, sw = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    f, nf = _per_dispatch(fdir, "FETCH_SIZE", kernel, per_call)
    w, nw = _per_dispatch(wdir, "WRITE_SIZE", kernel, per_call)
    fb, wb = f * 1024 * sf, w * 1024 * sw
    sha = kernel_source_sha()
    lines = [f"# HBM traffic of {kernel} ({key})", f"# commands: {command}", "",
             f"copy probe: FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB per {copy_bytes:.0f}-byte copy -> "
             f"scale fetch {sf:.3f}, write {sw:.3f}",
             (f"kernel: FETCH_SIZE {f:.0f} KiB, WRITE_SIZE {w:.0f} KiB per call "
              f"({nf} dispatches summed over {per_call} calls)" if per_call > 0 else
              f"kernel: FETCH_SIZE {f:.0f} KiB (median of {nf} dispatches), WRITE_SIZE {w:.0f} KiB ({nw})"),
             f"scaled bytes per {'call' if per_call > 0 else 'dispatch'}: read {fb:.4e}, write {wb:.4e}, "
             f"total {fb + wb:.4e}",
             f"kernel source sha256 {sha} (sweep.hip, sn_device.hpp, sn_kernels.hpp, build.py)"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))
    data = json.load(open(jpath)) if os.path.exists(jpath) else {}
    data[key] = {"bytes_per_launch": fb + wb, "read_bytes": fb, "write_bytes": wb, "kernel": kernel,
                 "kernel_src_sha256": sha, "fetch_scale": sf, "write_scale": sw}
    json.dump(data, open(jpath, "w"), indent=1)


def spans(d, kernel, per_call, out):
    rows = [r for r in csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_trace.csv"))))
            if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    per_call = int(per_call)
    lines = ["", f"# per call of {kernel} ({per_call} launches each, in launch order)",
             f"{'call':>5s} {'first start -> last end ms':>27s} {'summed durations ms':>20s} {'queues':>7s}"]
    for c in range(len(rows) // per_call):
        g = rows[c * per_call:(c + 1) * per_call]
        t0 = min(int(r["Start_Timestamp"]) for r in g)
        t1 = max(int(r["End_Timestamp"]) for r in g)
        tot = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in g)
        nq = len({r["Queue_Id"] for r in g})
        lines.append(f"{c:5d} {(t1 - t0) / 1e6:27.3f} {tot / 1e6:20.3f} {nq:7d}")
    open(out, "a").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(kernel, out, dirs, command):
    files = sources_of(kernel)
    names = ", ".join(os.path.basename(f) for f in files)
    lines = [f"# rocprofv3 counters of {kernel}, averaged per dispatch", f"# commands: {command}",
             f"# kernel source sha256 {kernel_source_sha(files)} ({names})", ""]
    for d in dirs.split(","):
        vals, disp = {}, {}
        for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
            if kernel not in r["Kernel_Name"]:
                continue
            c = r["Counter_Name"]
            vals[c] = vals.get(c, 0.0) + float(r["Counter_Value"])
            disp.setdefault(c, set()).add(r["Dispatch_Id"])
        for c in sorted(vals):
            lines.append(f"{os.path.basename(d.rstrip('/')):10s} {c:36s} {vals[c] / len(disp[c]):16.0f} "
                         f"per dispatch ({len(disp[c])} dispatches)")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "stats":
        stats(a[1], a[2], " ".join(a[3:]))
    elif a and a[0] == "spans":
        spans(a[1], a[2], a[3], a[4])
    elif a and a[0] == "counters":
        counters(a[1], a[2], a[3], " ".join(a[4:]))
    elif a and a[0] == "traffic":
        traffic(*a[1:10], " ".join(a[10:]))
    elif a and a[0] == "traffic_per_call":
        # traffic_per_call <calls> <key> <kernel> ... (as traffic)
        traffic(*a[2:11], " ".join(a[11:]), per_call=int(a[1]))
    else:
        raise SystemExit(__doc__)
