"""Summaries of rocprofv3 CSV output for the libmlu kernels.

Two reports, printed as short text that can be kept beside the numbers that
come from them:

  stats   <dir>                      per-kernel calls / total ms / average us
                                     from a `--kernel-trace --stats` run
  traffic --fetch <dir> --write <dir> --kernel REGEX --copy-bytes N --source F
          [--dispatches-per-step K]
                                     HBM bytes per dispatch of the kernels whose
                                     name matches REGEX, from two `--pmc` runs
                                     (FETCH_SIZE, then WRITE_SIZE, both in KiB
                                     per dispatch), each scaled by what the same
                                     counter reads for the calibration copy in
                                     that run (--copy-kernel REGEX), whose true
                                     traffic is N bytes read and N bytes written
  counters <dir> --kernel REGEX      mean of every collected counter per
                                     dispatch of the matching kernels
  timeline <dir> --main REGEX [--iter I ...]
                                     per outer iteration of the last traced
                                     factorization (one dispatch of the
                                     --main kernel on the caller's stream per
                                     iteration): its duration, the period to
                                     the next one, and the busy time and
                                     kernels of the other streams in between;
                                     with --iter, that iteration's kernels
  grid --calib <dir> --config LABEL:RUN_A:RUN_B:RUN_C ... --kernel REGEX ... --copy-bytes N
                                     per configuration and kernel: duration,
                                     matrix-core busy fraction, calibrated HBM
                                     bytes and their rate (run A: the MFMA
                                     counters of the calibration run and a
                                     kernel trace; run B: FETCH_SIZE; run C:
                                     WRITE_SIZE)
  mfma --calib <dir> --run <dir> --kernel REGEX [--kernel REGEX ...] [--source F]
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


def traffic(fetch_dir, write_dir, kernel, copy_bytes, source, copy_kernel, per_step=1):
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
    rec["dispatches_per_step"] = per_step
    rec["fetch_bytes_per_step"] = rec["fetch_bytes_per_launch"] * per_step
    rec["write_bytes_per_step"] = rec["write_bytes_per_launch"] * per_step
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


def trace_rows(d: str):
    """Kernel dispatches of a --kernel-trace run: dicts with name, queue,
    start / end (ns) and grid size, sorted by start."""
    rows = []
    with open(_find(d, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            rows.append({"name": short_name(_col(r, "Kernel_Name")), "queue": _col(r, "Queue_Id"),
                         "s": int(_col(r, "Start_Timestamp")), "e": int(_col(r, "End_Timestamp")),
                         "grid": int(_col(r, "Grid_Size_X"))})
    rows.sort(key=lambda r: r["s"])
    return rows


def timeline(d, main_regex, per_fact, min_grid, show):
    rows = [r for r in trace_rows(d) if "mlu::" in r["name"]]
    main = [r for r in rows if re.search(main_regex, r["name"]) and r["grid"] >= min_grid]
    if len(main) < per_fact:
        raise RuntimeError("fewer main dispatches than one factorization")
    fac = main[-per_fact:]
    mq = fac[0]["queue"]
    print(f"{'iter':>4s} {'main_us':>8s} {'period_us':>9s} {'other_busy_us':>13s} {'other_kernels':>13s}")
    total = 0.0
    for i in range(len(fac) - 1):
        a, b = fac[i], fac[i + 1]
        other = [x for x in rows if x["queue"] != mq and a["s"] <= x["s"] < b["s"]]
        busy = sum(x["e"] - x["s"] for x in other) / 1e3
        total += (b["s"] - a["s"]) / 1e3
        print(f"{i:4d} {(a['e'] - a['s']) / 1e3:8.0f} {(b['s'] - a['s']) / 1e3:9.0f} {busy:13.0f} {len(other):13d}")
    print(f"sum of periods: {total / 1e3:.2f} ms")
    for i in show:
        a, b = fac[i], fac[i + 1]
        per = defaultdict(lambda: [0, 0.0])
        for x in rows:
            if a["s"] <= x["s"] < b["s"]:
                key = ("main" if x["queue"] == mq else "other", x["name"])
                per[key][0] += 1
                per[key][1] += (x["e"] - x["s"]) / 1e3
        print(f"iteration {i}: stream, kernel, launches, total us")
        for (q, k), (c, t) in sorted(per.items()):
            print(f"  {q:5s} {k:40s} {c:4d} {t:9.1f}")


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


def _durations(d: str):
    """{dispatch_id: duration in ns} from the kernel trace of a run."""
    out = {}
    with open(_find(d, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            did = int(_col(r, "Dispatch_Id", "Dispatch-Id"))
            out[did] = int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))
    return out


def grid(calib_dir, configs, kernels, copy_bytes, copy_kernel, calib_kernel="k_mfma_peak"):
    """Per configuration and kernel: dispatches, average duration, matrix-core
    busy fraction (normalized as in `mfma`, run A collecting the same counters
    as the calibration run), calibrated HBM bytes per dispatch (FETCH_SIZE
    from run B, WRITE_SIZE from run C, each scaled by the copy calibration of
    its own run) and the rate those bytes make over the duration.  `configs`:
    (label, run A with the MFMA counters and a kernel trace, run B, run C)."""
    n_c, cal = counters(calib_dir, calib_kernel)
    if n_c == 0:
        raise RuntimeError(f"no {calib_kernel} dispatch in {calib_dir}")
    cal_rate = cal["SQ_VALU_MFMA_BUSY_CYCLES"] / cal["GRBM_GUI_ACTIVE"]
    rows = []
    for label, da, db, dc in configs:
        disp_a, disp_b, disp_c, dur = per_dispatch(da), per_dispatch(db), per_dispatch(dc), _durations(da)
        fscale = copy_bytes / (_copy_dispatch(disp_b, "FETCH_SIZE", copy_kernel)[1] * 1024.0)
        wscale = copy_bytes / (_copy_dispatch(disp_c, "WRITE_SIZE", copy_kernel)[1] * 1024.0)
        for k in kernels:
            ids = [i for i, (name, v) in disp_a.items() if re.search(k, name) and v.get("GRBM_GUI_ACTIVE")]
            fv = [v["FETCH_SIZE"] for name, v in disp_b.values() if re.search(k, name) and "FETCH_SIZE" in v]
            wv = [v["WRITE_SIZE"] for name, v in disp_c.values() if re.search(k, name) and "WRITE_SIZE" in v]
            if not ids or not fv or not wv:
                continue
            # time-weighted: busy cycles over active cycles summed over the
            # dispatches (a dispatch that finds no work weighs nothing)
            busy = sum(disp_a[i][1]["SQ_VALU_MFMA_BUSY_CYCLES"] for i in ids) / \
                sum(disp_a[i][1]["GRBM_GUI_ACTIVE"] for i in ids) / cal_rate
            flops = 512.0 * sum(disp_a[i][1].get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for i in ids) / len(ids)
            fetch = sum(fv) / len(fv) * 1024.0 * fscale
            write = sum(wv) / len(wv) * 1024.0 * wscale
            ns = [dur[i] for i in ids if i in dur]
            t = sum(ns) / len(ns) if ns else float("nan")
            rows.append({"config": label, "kernel": k, "dispatches": len(ids), "avg_us": round(t / 1e3, 2),
                         "mfma_busy_frac": round(busy, 4), "f64_gflop": round(flops / 1e9, 4),
                         "fetch_bytes": round(fetch), "write_bytes": round(write),
                         "hbm_gbs": round((fetch + write) / t, 1) if ns else None})
    return rows


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
    t.add_argument("--dispatches-per-step", type=int, default=1,
                   help="dispatches of the kernel per unit of the traced launch (RU2 and its helpers: 2)")
    t.add_argument("--copy-kernel", default=r"AUnaryFunctor<double, double, double, .*MulFunctor",
                   help="regex naming the calibration copy (bench.py --copy-calibration runs x * 1.0)")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    tl = sub.add_parser("timeline")
    tl.add_argument("dir")
    tl.add_argument("--main", required=True, help="regex of the kernel launched once per iteration")
    tl.add_argument("--per-factorization", type=int, default=62)
    tl.add_argument("--min-grid", type=int, default=64 * 256 + 1,
                    help="grid size (threads) above which a dispatch counts as the main one")
    tl.add_argument("--iter", type=int, action="append", default=[])
    mm = sub.add_parser("mfma")
    mm.add_argument("--calib", required=True)
    mm.add_argument("--run", required=True)
    mm.add_argument("--kernel", action="append", required=True)
    mm.add_argument("--source", default=None, help="kernel source whose sha1 the record carries")
    g = sub.add_parser("grid")
    g.add_argument("--calib", required=True)
    g.add_argument("--config", action="append", required=True, metavar="LABEL:RUN_A:RUN_B:RUN_C")
    g.add_argument("--kernel", action="append", required=True)
    g.add_argument("--copy-bytes", type=int, required=True)
    g.add_argument("--copy-kernel", default=r"AUnaryFunctor<double, double, double, .*MulFunctor")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(f"{'kernel':72s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
        for name, calls, tot, avg, pct in kernel_stats(a.dir)[: a.top]:
            print(f"{name:72s} {calls:7d} {tot / 1e6:10.3f} {avg / 1e3:10.3f} {pct:6.2f}")
    elif a.cmd == "traffic":
        rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.source, a.copy_kernel, a.dispatches_per_step)
        for k, v in rec.items():
            print(f"{k}: {v}")
        print("TRAFFIC_JSON: " + json.dumps(rec))
    elif a.cmd == "timeline":
        timeline(a.dir, a.main, a.per_factorization, a.min_grid, a.iter)
    elif a.cmd == "grid":
        cfgs = [tuple(c.split(":")) for c in a.config]
        rows = grid(a.calib, cfgs, a.kernel, a.copy_bytes, a.copy_kernel)
        print("| config | kernel | dispatches | avg us | MFMA busy | GFLOP (counted) | MB read | MB written | GB/s |")
        print("|---|---|---|---|---|---|---|---|---|")
        for r in rows:
            print(f"| {r['config']} | {r['kernel']} | {r['dispatches']} | {r['avg_us']} | "
                  f"{100 * r['mfma_busy_frac']:.1f}% | {r['f64_gflop']} | {r['fetch_bytes'] / 1e6:.1f} | "
                  f"{r['write_bytes'] / 1e6:.1f} | {r['hbm_gbs']} |")
        print("GRID_JSON: " + json.dumps(rows))
    elif a.cmd == "mfma":
        rec = mfma(a.calib, a.run, a.kernel)
        if a.source:
            rec["source_sha1"] = hashlib.sha1(open(a.source, "rb").read()).hexdigest()
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
