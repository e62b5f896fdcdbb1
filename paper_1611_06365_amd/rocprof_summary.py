"""Summaries of rocprofv3 CSV output for the libmlu kernels.

Two reports, printed as short text that can be kept beside the numbers that
come from them:

  stats   <dir>                      per-kernel calls / total ms / average us
                                     from a `--kernel-trace --stats` run
  traffic --fetch <dir> --write <dir> --kernel REGEX --copy-bytes N --source F
                                     HBM bytes per dispatch of the kernels whose
                                     name matches REGEX, from two `--pmc` runs
                                     (FETCH_SIZE, then WRITE_SIZE, both in KiB
                                     per dispatch), each scaled by what the same
                                     counter reads for the calibration copy in
                                     that run (--copy-kernel REGEX), whose true
                                     traffic is N bytes read and N bytes written
  counters <dir> --kernel REGEX      mean of every collected counter per
                                     dispatch of the matching kernels
  mfma --calib <dir> --run <dir> --kernel REGEX [--kernel REGEX ...]
                                     matrix-core utilization of the matching
                                     kernels: SQ_VALU_MFMA_BUSY_CYCLES per
                                     GRBM_GUI_ACTIVE cycle of each, over the
                                     same ratio for the calibration kernel
                                     (k_mfma_peak, every SIMD's matrix unit
                                     kept busy), and the FP64 flops per cycle
                                     from SQ_INSTS_VALU_MFMA_MOPS_F64 (x 512)

Run with `--output-format csv`; the CSV files are searched for under <dir>.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def _col(row: dict, *names: str):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)[:72]


def kernel_stats(d: str):
    rows = []
    with open(_find(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(_col(r, "Name", "KernelName")), int(_col(r, "Calls")),
                         float(_col(r, "TotalDurationNs")), float(_col(r, "AverageNs")),
                         float(_col(r, "Percentage"))))
    rows.sort(key=lambda x: -x[2])
    return rows


def per_dispatch(d: str):
    """{dispatch_id: (kernel_name, {counter: value})} from a --pmc run."""
    out = {}
    with open(_find(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            did = int(_col(r, "Dispatch_Id", "Dispatch-Id"))
            name = _col(r, "Kernel_Name", "Kernel-Name")
            cname = _col(r, "Counter_Name", "Counter-Name")
            val = float(_col(r, "Counter_Value", "Counter-Value"))
            ent = out.setdefault(did, (name, defaultdict(float)))
            ent[1][cname] += val
    return out


def _copy_dispatch(disp, counter, pattern):
    """The dispatch whose name matches `pattern` with the largest reading of
    `counter`: the 1 GiB copy that the profiled program runs for calibration."""
    best = None
    for name, vals in disp.values():
        if re.search(pattern, name) and counter in vals:
            if best is None or vals[counter] > best[1]:
                best = (name, vals[counter])
    if best is None:
        raise RuntimeError("no copy-like calibration dispatch in the counter run")
    return best


def traffic(fetch_dir, write_dir, kernel, copy_bytes, source, copy_kernel):
    rec = {"kernel_regex": kernel, "copy_bytes": copy_bytes, "copy_kernel_regex": copy_kernel}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = per_dispatch(d)
        cname, cval = _copy_dispatch(disp, counter, copy_kernel)
        scale = copy_bytes / (cval * 1024.0)
        vals = [v[counter] for n, v in disp.values() if re.search(kernel, n) and counter in v]
        if not vals:
            raise RuntimeError(f"no dispatch of {kernel} in {d}")
        mean_kib = sum(vals) / len(vals)
        rec[f"{key}_dispatches"] = len(vals)
        rec[f"{key}_kib_per_dispatch_raw"] = round(mean_kib, 1)
        rec[f"{key}_copy_kernel"] = short_name(cname)
        rec[f"{key}_copy_kib_raw"] = round(cval, 1)
        rec[f"{key}_scale"] = round(scale, 5)
        rec[f"{key}_bytes_per_launch"] = round(mean_kib * 1024.0 * scale)
    rec["source_sha1"] = hashlib.sha1(open(source, "rb").read()).hexdigest()
    return rec


def counters(d, kernel):
    disp = per_dispatch(d)
    acc, cnt = defaultdict(float), 0
    for name, vals in disp.values():
        if re.search(kernel, name):
            cnt += 1
            for k, v in vals.items():
                acc[k] += v
    return cnt, {k: v / max(cnt, 1) for k, v in acc.items()}


def mfma(calib_dir, run_dir, kernels, calib_kernel="k_mfma_peak"):
    """Utilization of the matrix units per kernel, normalized by the
    calibration kernel's busy-cycle rate."""
    n_c, cal = counters(calib_dir, calib_kernel)
    if n_c == 0:
        raise RuntimeError(f"no {calib_kernel} dispatch in {calib_dir}")
    cal_rate = cal["SQ_VALU_MFMA_BUSY_CYCLES"] / cal["GRBM_GUI_ACTIVE"]
    cal_fpc = 512.0 * cal["SQ_INSTS_VALU_MFMA_MOPS_F64"] / cal["GRBM_GUI_ACTIVE"]
    out = {"calibration": {"kernel": calib_kernel, "dispatches": n_c,
                           "mfma_busy_per_gui_cycle": round(cal_rate, 3),
                           "f64_flops_per_gui_cycle": round(cal_fpc, 1)}, "kernels": {}}
    for k in kernels:
        n, m = counters(run_dir, k)
        if n == 0 or not m.get("GRBM_GUI_ACTIVE"):
            continue
        rate = m["SQ_VALU_MFMA_BUSY_CYCLES"] / m["GRBM_GUI_ACTIVE"]
        fpc = 512.0 * m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) / m["GRBM_GUI_ACTIVE"]
        out["kernels"][k] = {"dispatches": n, "mfma_busy_frac": round(rate / cal_rate, 4),
                             "f64_flops_frac_of_calibration": round(fpc / cal_fpc, 4),
                             "gui_active_cycles_per_dispatch": round(m["GRBM_GUI_ACTIVE"]),
                             "mfma_mops_f64_per_dispatch": m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)}
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=16)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--copy-kernel", default=r"AUnaryFunctor<double, double, double, .*MulFunctor",
                   help="regex naming the calibration copy (bench.py --copy-calibration runs x * 1.0)")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    mm = sub.add_parser("mfma")
    mm.add_argument("--calib", required=True)
    mm.add_argument("--run", required=True)
    mm.add_argument("--kernel", action="append", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(f"{'kernel':72s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
        for name, calls, tot, avg, pct in kernel_stats(a.dir)[: a.top]:
            print(f"{name:72s} {calls:7d} {tot / 1e6:10.3f} {avg / 1e3:10.3f} {pct:6.2f}")
    elif a.cmd == "traffic":
        rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.source, a.copy_kernel)
        for k, v in rec.items():
            print(f"{k}: {v}")
        print("TRAFFIC_JSON: " + json.dumps(rec))
    elif a.cmd == "mfma":
        rec = mfma(a.calib, a.run, a.kernel)
        print(json.dumps(rec, indent=1))
        print("MFMA_JSON: " + json.dumps(rec))
    else:
        n, means = counters(a.dir, a.kernel)
        print(f"dispatches matching {a.kernel}: {n}")
        for k in sorted(means):
            print(f"{k}: {means[k]:.6g}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
