"""Summaries of rocprofv3 output for the kernels of this package.

    python -m paper_2203_02479_amd.profsum stats DIR
        per-kernel calls / average / total time from a --kernel-trace --stats run,
        then per (kernel, grid size) the launch count and median duration
    python -m paper_2203_02479_amd.profsum pmc DIR COUNTER [--last N]
        per-kernel mean of COUNTER over the last N dispatches of each kernel
        (a --pmc run; FETCH_SIZE / WRITE_SIZE are KiB per dispatch)
    python -m paper_2203_02479_amd.profsum traffic FETCH_DIR WRITE_DIR CALIB_FETCH_DIR CALIB_WRITE_DIR
        HBM bytes per launch of each bench stage, each counter scaled by what
        it reads for a plain device copy of known size (bench.py --calib),
        printed as JSON for bench.py --traffic

DIR is searched recursively for the CSV files rocprofv3 writes.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import re
import statistics
import sys

# bench stage -> kernel name pattern of the timed single-plane step
STAGE_KERNELS = {
    "fill": r"k_fill_zero\b",
    "raster": r"k_raster<[0-2][,>]",
    "r2c": r"k_r2c_rows",
    "wire": r"k_wire_fused|k_wire_static",
    "c2r": r"k_c2r_rows",
}
CALIB_BYTES = 4 * (1 << 28)          # bench.py --calib copies 1 GiB of float32
# source files each stage's kernels are built from: a stored traffic figure
# holds only while their contents are unchanged
STAGE_SOURCES = {
    "fill": ("fft_kernels.hip", "lar_internal.hpp"),
    "raster": ("raster_kernels.hip", "lar_internal.hpp"),
    "r2c": ("fft_kernels.hip", "lar_internal.hpp"),
    "wire": ("fft_kernels.hip", "lar_internal.hpp"),
    "c2r": ("fft_kernels.hip", "lar_internal.hpp"),
}


def source_digest(stage):
    import hashlib
    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in STAGE_SOURCES[stage]:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def _short(name):
    name = re.sub(r"\(.*$", "", name)          # drop the argument list
    name = name.replace("void ", "").replace("lar::", "")
    return name


def stats(d):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append((_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                    float(r["TotalDurationNs"]) / 1e6))
    return out


def launch_medians(d):
    """{(kernel, grid size): (launches, median us)} from the kernel trace:
    launches of one kernel with different grids (different row counts,
    batch sizes) are kept apart, and the median is not moved by the first,
    cold launch the way the average is."""
    try:
        path = _find(d, "kernel_trace.csv")
    except FileNotFoundError:
        return {}
    per = {}
    for r in csv.DictReader(open(path)):
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        key = (_short(r["Kernel_Name"]), int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0))
        per.setdefault(key, []).append(us)
    return {k: (len(v), statistics.median(v)) for k, v in per.items()}


def _pmc_rows(d, counter):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        k = _short(r["Kernel_Name"])
        per.setdefault(k, []).append((int(r.get("Dispatch_Id", 0)), float(r["Counter_Value"])))
    for v in per.values():
        v.sort()
    return per


def pmc(d, counter, last=2):
    """{kernel: mean counter value over its last `last` dispatches}."""
    return {k: statistics.mean(x for _, x in v[-last:]) for k, v in _pmc_rows(d, counter).items()}


def last_dispatched(d, counter, pattern):
    """The kernel matching pattern that was dispatched last (the instantiation
    the timed steps at the end of the run used)."""
    best, when = None, -1
    for k, v in _pmc_rows(d, counter).items():
        if re.search(pattern, k) and v[-1][0] > when:
            best, when = k, v[-1][0]
    return best


def _copy_value(m):
    """The counter of the largest copy-like kernel of the calibration run."""
    cands = {k: v for k, v in m.items() if re.search(r"copy|Copy|elementwise", k)}
    if not cands:
        cands = m
    return max(cands.values())


def traffic(fd, wd, cfd, cwd):
    f, w = pmc(fd, "FETCH_SIZE"), pmc(wd, "WRITE_SIZE")
    cf, cw = _copy_value(pmc(cfd, "FETCH_SIZE", last=3)), _copy_value(pmc(cwd, "WRITE_SIZE", last=3))
    # KiB per dispatch -> bytes, then scaled so the copy reads/writes its own size
    kf = CALIB_BYTES / (cf * 1024.0)
    kw = CALIB_BYTES / (cw * 1024.0)
    out = {"_calibration": {"copy_bytes": CALIB_BYTES, "fetch_kib": cf, "write_kib": cw,
                            "fetch_scale": kf, "write_scale": kw}}
    for stage, pat in STAGE_KERNELS.items():
        k = last_dispatched(fd, "FETCH_SIZE", pat)
        if k is None:
            continue
        rd = f[k] * 1024.0 * kf
        wr = w.get(k, 0.0) * 1024.0 * kw
        out[stage] = {"kernel": k, "read_bytes": round(rd), "write_bytes": round(wr),
                      "bytes": round(rd + wr), "source": source_digest(stage)}
    return out


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    cmd = argv[0]
    if cmd == "stats":
        print(f"{'calls':>6} {'avg_us':>10} {'total_ms':>10}  kernel")
        for name, calls, avg, tot in sorted(stats(argv[1]), key=lambda r: -r[3]):
            print(f"{calls:6d} {avg:10.2f} {tot:10.3f}  {name}")
        med = launch_medians(argv[1])
        if med:
            print(f"\nper launch shape (grid threads): launches, median us")
            for (name, grid), (n, m) in sorted(med.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
                print(f"{n:6d} {m:10.2f} {grid:10d}  {name}")
    elif cmd == "pmc":
        last = 2
        if "--last" in argv:
            last = int(argv[argv.index("--last") + 1])
        for k, v in sorted(pmc(argv[1], argv[2], last).items(), key=lambda kv: -kv[1]):
            print(f"{v:16.1f}  {k}")
    elif cmd == "traffic":
        print(json.dumps(traffic(*argv[1:5]), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
