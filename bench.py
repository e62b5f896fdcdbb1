#!/usr/bin/env python3
"""Benchmark: FP64 blocked LU with partial pivoting on one MI355X.

A step is one whole factorization P A = L U of an n x n matrix (every step of
the hot path: panel factorizations, row interchanges, triangular solves and
trailing updates) through the C ABI.  Inputs are synthetic and seeded:
A = B B^T + n I with B ~ N(0, 1) (default) or U(0, 1) entries, generated on the
GPU; one pristine copy per step is resident in HBM before the timed region, so
the timed region contains factorizations only.

Prints ONE JSON line.  `value` is GFLOP/s = (2 n^3 / 3) / (seconds per step).
`roofline` covers the dominant kernel (the outer trailing-update GEMM), timed
with HIP events around each of its launches inside the timed region.
`cpu_baseline` times the plain C oracle on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GFLOP/s & %MFMA roofline at n=16384 (FP64 vs mixed+refine @1e-13); batched ops/s"
FP64_PEAK_TFLOPS = 78.6
# the traced launches: the outer trailing updates carrying nearly all flops
KERNEL_LABEL = {
    "la": "k_gemm_queue_whole (RU2 as a persistent tile queue on the CUs the panel stream leaves, pipelined across "
          "tiles, joined by the panel's workgroups after PF3; the last iteration's k_gemm_trailing), "
          "v_mfma_f64_16x16x4f64",
    "rl": "k_gemm_trailing (RL3), v_mfma_f64_16x16x4f64",
    "ll": "k_gemm_trailing (LL2), v_mfma_f64_16x16x4f64",
}
TRAFFIC_KERNEL = {"la": "k_gemm_queue_whole", "rl": "k_gemm_trailing", "ll": "k_gemm_trailing"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_queue_whole_la_n16384_traffic.md")
MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_counters_la_n16384.md")
GEMM_SRC = os.path.join(ROOT, "paper_1611_06365_amd", "csrc", "gemm.hip")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sampled_residual(A, F, ipiv, nsamp=512, seed=0):
    """max |(P A)[i,j] - sum_k L[i,k] U[k,j]| / max|A| over random (i, j)."""
    import numpy as np
    import torch

    n = A.shape[0]
    piv = ipiv.cpu().numpy().astype(np.int64) - 1
    perm = np.arange(n)
    for c in range(n):
        p = piv[c]
        perm[c], perm[p] = perm[p], perm[c]
    rng = np.random.default_rng(seed)
    ii = torch.from_numpy(rng.integers(0, n, nsamp)).to(A.device)
    jj = torch.from_numpy(rng.integers(0, n, nsamp)).to(A.device)
    pa = A[torch.from_numpy(perm).to(A.device)[ii], jj]
    Lrows = F[ii, :].clone()
    Ucols = F[:, jj].T.clone()
    k = torch.arange(n, device=A.device)
    Lrows = torch.where(k[None, :] < ii[:, None], Lrows, torch.zeros_like(Lrows))
    Lrows[torch.arange(nsamp, device=A.device), ii] = 1.0
    Ucols = torch.where(k[None, :] <= jj[:, None], Ucols, torch.zeros_like(Ucols))
    lu = (Lrows * Ucols).sum(dim=1)
    return float((pa - lu).abs().max() / A.abs().max())


def traffic_record():
    """Per-launch HBM bytes of the trailing GEMM from the committed rocprofv3
    counter summary, or None if missing or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    m = re.search(r"TRAFFIC_JSON:\s*(\{.*\})", open(TRAFFIC_FILE).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    sha = hashlib.sha1(open(GEMM_SRC, "rb").read()).hexdigest()
    if rec.get("source_sha1") != sha:
        return None
    return rec


def mfma_record():
    """RU2's matrix-core busy fraction from the committed counter summary, or
    None if missing or taken on a different kernel source."""
    if not os.path.exists(MFMA_FILE):
        return None
    m = re.search(r"MFMA_JSON:\s*(\{.*\})", open(MFMA_FILE).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha1") != hashlib.sha1(open(GEMM_SRC, "rb").read()).hexdigest():
        return None
    return rec


def cpu_baseline(n: int):
    import numpy as np

    import inputs
    from oracle import c_oracle

    c_oracle.build(force=False)
    A = inputs.spd_bbt(n, seed=0)
    # threads: the OpenMP team the oracle runs with (OMP_NUM_THREADS, the CPU
    # share given to this GPU where one is set), else every CPU this process
    # may run on
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = int(os.environ.get("OMP_NUM_THREADS", avail))
    t0 = time.perf_counter()
    ipiv, info = c_oracle.dgetrf_rl(A, nb=64)
    dt = time.perf_counter() - t0
    return {
        "value": round((2.0 * n ** 3 / 3.0) / dt / 1e9, 3),
        "unit": "GFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"plain C blocked-RL oracle (nb=64, OpenMP, {cores} threads) factoring one n={n} A=B B^T+nI "
                  f"matrix (seed 0) in {dt:.2f} s: a bounded sample of the n=16384 workload, which has "
                  f"~{(16384 / n) ** 3:.0f}x the flops (rate in GFLOP/s of that sample)",
        "cpu_model": cpu_model(),
        "host_logical_cpus": os.cpu_count(),
        "cpus_available_to_process": avail,
        "info": info,
    }


def cpu_model() -> str | None:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def uniform_section(args, dev, work, ipiv, info):
    """The paper's own workload: look-ahead LU (the bench's variant and block
    sizes) on an n x n matrix with U(0, 1) entries (seed 0), where partial
    pivoting interchanges rows at nearly every column.  One warm-up, then the
    best of two factorizations of fresh copies (restored outside the timed
    region), HIP events."""
    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    n = args.n
    A = D.uniform01(n, seed=0, device=dev)
    M = torch.empty_like(A)
    times = []
    for r in range(3):
        M.copy_(A)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mlu.getrf(M, variant=args.variant, nb=args.nb, nb_inner=args.nb_inner, inner=args.inner, ipiv=ipiv,
                  info=info, work=work)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    ms = min(times)
    gf = 2.0 * n ** 3 / 3.0 / (ms / 1e3) / 1e9
    swaps = int((ipiv.cpu() != torch.arange(1, n + 1, dtype=torch.int32)).sum().item())
    out = {"workload": f"getrf FP64 n={n} U(0,1) (seed 0), variant={args.variant.upper()}, nb={args.nb}, "
                       f"nb_inner={args.nb_inner}, inner={args.inner.upper()}",
           "ms": round(ms, 3), "gflops": round(gf, 1), "frac_fp64_peak": round(gf / (FP64_PEAK_TFLOPS * 1e3), 4),
           "info": int(info.item()), "interchanges": swaps, "sampled_residual": sampled_residual(A, M, ipiv)}
    log(f"uniform: {out}")
    del A, M
    torch.cuda.empty_cache()
    return out


def batched_section(args, dev):
    """`args.batch` independent matrices, orders n ~ U{8..512} (seed 0), each
    A = B B^T + n I with B ~ N(0, 1), factored by one mlu_?getrf_batched call
    (FP64 and FP32), eager and as a captured graph replay; a pristine copy is
    restored outside the timed region.  The panel width is chosen first by
    mlu.tune_batched (each candidate timed on copies).  matrices/s and
    GFLOP/s = sum(2n^3/3)/t."""
    import numpy as np
    import torch

    from paper_1611_06365_amd import mlu

    rng = np.random.default_rng(0)
    ns = rng.integers(8, 513, args.batch)
    flops = float(np.sum(2.0 * ns.astype(np.float64) ** 3 / 3.0))
    out = {"batch": int(args.batch), "n_range": [8, 512],
           "matrix": "A = B B^T + n I, B ~ N(0,1) per matrix" + (" (host-built)" if args.batch_host_inputs else ""),
           "gflop": round(flops / 1e9, 3)}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        log(f"batched {name}: generating {args.batch} matrices")
        offs = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)])
        buf = torch.empty(int(offs[-1]), dtype=dt, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(1)
        hg = np.random.default_rng(1)
        for n in np.unique(ns):
            idx = np.nonzero(ns == n)[0]
            if args.batch_host_inputs:   # no vendor GEMM in the process (counter runs)
                hb = hg.standard_normal((len(idx), int(n), int(n)))
                a = torch.from_numpy(hb @ hb.transpose(0, 2, 1)).to(dev)
                del hb
            else:
                b = torch.randn(len(idx), int(n), int(n), generator=g, dtype=torch.float64, device=dev)
                a = torch.bmm(b, b.transpose(1, 2).contiguous())
                del b
            a.diagonal(dim1=1, dim2=2).add_(float(n))
            for t, i in enumerate(idx):
                buf[int(offs[i]):int(offs[i + 1])].copy_(a[t].reshape(-1))
            del a
        pristine = buf.clone()
        mats = [buf[int(offs[i]):int(offs[i + 1])].view(int(n), int(n)) for i, n in enumerate(ns)]
        torch.cuda.synchronize()
        nb, tune_ms = mlu.tune_batched(mats, max_n=512)
        log(f"batched {name}: panel width by timing {tune_ms} -> {nb}")
        plan = mlu.BatchPlan(mats, max_n=512, nb=nb)
        torch.cuda.synchronize()

        def once(run):
            buf.copy_(pristine)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)

        once(plan.run)
        t_eager = min(once(plan.run) for _ in range(3))
        bad = int((plan.info != 0).sum().item())
        s = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                plan.run(stream=s)
        t_graph = min(once(graph.replay) for _ in range(3))
        out[name] = {"nb": nb, "tuning_ms": {str(k): round(v, 3) for k, v in tune_ms.items()},
                     "ms": round(t_eager, 3), "ms_graph_replay": round(t_graph, 3),
                     "matrices_per_s": round(args.batch / (t_eager / 1e3), 1),
                     "gflops": round(flops / (t_eager / 1e3) / 1e9, 1), "nonzero_info": bad}
        log(f"batched {name}: {out[name]}")
        del plan, mats, buf, pristine, graph
        torch.cuda.empty_cache()
    return out


def et_section(args, A, ipiv, info, work):
    """Look-ahead LU with early termination of the panel (mlu_dgetrf_et) beside
    plain look-ahead (mlu_dgetrf, LA) on the bench matrix: the left-looking
    panel without stopping (force=never), then with the flag, for two planned
    widths and minimum stop widths.  Each run factors a fresh copy of A
    (restored outside the timed region), timed with HIP events; the best of two
    runs.  ET waits on the device once per outer iteration, inside its timed
    region."""
    import torch

    from paper_1611_06365_amd import mlu

    M = torch.empty_like(A)
    widths = {}

    def timed(fn, reps=2):
        best = None
        for _ in range(reps + 1):   # the first is a warm-up
            M.copy_(A)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    rows = []
    la_ms = {}
    for nb, min_width, force in ((256, 0, "never"), (256, 0, "signal"), (256, 128, "signal"), (512, 256, "signal")):
        if nb not in la_ms:
            la_ms[nb] = timed(lambda: mlu.getrf(M, variant="la", nb=nb, nb_inner=args.nb_inner, ipiv=ipiv,
                                                info=info, work=work))
        ok_la = int(info.item())

        def et():
            widths["w"] = mlu.getrf_et(M, nb=nb, nb_inner=args.nb_inner, force=force, min_width=min_width,
                                       ipiv=ipiv, info=info, work=work)[2]

        t_et = timed(et)
        w = widths["w"]
        row = {"nb": nb, "min_width": min_width, "force": force, "ms_la": round(la_ms[nb], 3),
               "ms_la_et": round(t_et, 3),
               "info": [ok_la, int(info.item())],
               "panels": len(w), "width_min": min(w), "width_max": max(w), "width_mean": round(sum(w) / len(w), 1),
               "stopped_early": sum(1 for x in w[1:-1] if x < nb)}
        log(f"ET nb={nb} min_width={min_width} force={force}: {row}")
        rows.append(row)
    del M
    return {"what": "look-ahead with early termination of the left-looking panel (flag raised when RU2 "
                    "completes; the panel stops after its current 16-column block and the next block size is "
                    "the width it reached) vs plain look-ahead (RL inner panel)",
            "n": A.shape[0], "matrix": args.matrix, "rows": rows}


def ws_section(args, A, ipiv, info, work):
    """Worker sharing on and off (the comparison of the paper's Section 5.2):
    look-ahead (mlu_dgetrf, LA: the panel's workgroups join RU2's tile queue
    once PF3 is done) against MLU_LA_NOWS (they idle after PF3), on the bench
    matrix; the best of three runs after a warm-up, each on a fresh copy."""
    import torch

    from paper_1611_06365_amd import mlu

    M = torch.empty_like(A)

    def timed(variant, reps=3):
        best = None
        for _ in range(reps + 1):   # the first is a warm-up
            M.copy_(A)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mlu.getrf(M, variant=variant, nb=args.nb, nb_inner=args.nb_inner, ipiv=ipiv, info=info, work=work)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best, int(info.item())

    t_ws, i_ws = timed("la")
    t_no, i_no = timed("la_nows")
    del M
    out = {"what": "look-ahead with worker sharing (LA) vs without (the panel stream idles after PF3)",
           "n": A.shape[0], "nb": args.nb, "matrix": args.matrix, "ms_la": round(t_ws, 3),
           "ms_la_without_worker_sharing": round(t_no, 3), "gain": round(t_no / t_ws, 4), "info": [i_ws, i_no]}
    log(f"worker sharing: {out}")
    return out


def lead_schedule(n: int, nb: int):
    """Blocks of 2 nb over the first 3/8 of the order (then nb)."""
    return [2 * nb] * max(1, (3 * n // 8) // (2 * nb))


def schedule_section(args, A, ipiv, info, work):
    """The block size chosen per iteration (the "determine block size" step of
    the loop): the bench's variant with blocks of 2 nb over the first 3/8 of the
    order, then nb, beside constant nb, on the bench matrix.  Each run factors a
    fresh copy of A (restored outside the timed region); the two forms
    alternate, best of three each after a warm-up.  Not the headline figure,
    whose workload fixes nb."""
    import torch

    from paper_1611_06365_amd import mlu

    n = A.shape[0]
    sched = lead_schedule(n, args.nb)
    lead, count = sched[0], len(sched)
    M = torch.empty_like(A)

    def run(schedule):
        M.copy_(A)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mlu.getrf(M, variant=args.variant, nb=args.nb, nb_inner=args.nb_inner, schedule=schedule, ipiv=ipiv,
                  info=info, work=work)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(None)
    run(sched)
    const_ms, sched_ms = [], []
    for _ in range(3):
        const_ms.append(run(None))
        sched_ms.append(run(sched))
    out = {"what": f"{args.variant.upper()} with {count} blocks of {lead} then {args.nb}, vs constant nb={args.nb}",
           "schedule": sched, "nb_after": args.nb,
           "ms_constant": round(min(const_ms), 3), "ms_schedule": round(min(sched_ms), 3),
           "gflops_schedule": round(2.0 * n ** 3 / 3.0 / (min(sched_ms) / 1e3) / 1e9, 1),
           "speedup": round(min(const_ms) / min(sched_ms), 4),
           "info": int(info.item()), "sampled_residual": sampled_residual(A, M, ipiv)}
    log(f"schedule: {out}")
    del M
    return out


def grid_section(args, dev):
    """Every variant at n in {4096, 8192, 16384} and nb in {64, 128, 256} (b_i =
    16) on A = B B^T + n I (seed 0): one warm-up, then the best of two timed
    factorizations (HIP events), each on a fresh copy restored outside the
    timed region."""
    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    rows = []
    work = mlu.workspace(dev)
    for n in (4096, 8192, 16384):
        A = D.spd_bbt(n, seed=0, device=dev)
        M = torch.empty_like(A)
        ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        for variant in ("rl", "ll", "la"):
            for nb in (64, 128, 256):
                best = None
                for r in range(3):
                    M.copy_(A)
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    mlu.getrf(M, variant=variant, nb=nb, nb_inner=16, ipiv=ipiv, info=info, work=work)
                    e1.record()
                    torch.cuda.synchronize()
                    if r > 0:
                        t = e0.elapsed_time(e1)
                        best = t if best is None else min(best, t)
                gf = 2.0 * n ** 3 / 3.0 / (best / 1e3) / 1e9
                row = {"n": n, "variant": variant, "nb": nb, "ms": round(best, 3), "gflops": round(gf, 1),
                       "frac_fp64_peak": round(gf / (FP64_PEAK_TFLOPS * 1e3), 4), "info": int(info.item())}
                log(f"grid: {row}")
                rows.append(row)
        del A, M
        torch.cuda.empty_cache()
    return rows


def selector_section(args):
    """The learned selector: its choice for the bench workload, its inference
    latency through the C ABI (mlu_select) and in Python, and the regret on
    the held-out orders from the committed training report."""
    from paper_1611_06365_amd import mlu
    from paper_1611_06365_amd import selector as S

    if not os.path.exists(S.MODEL_PATH):
        return None
    choice = mlu.select(args.n, "fp64", with_fallback=True)
    choice_batched = mlu.select(256, "fp64", batch=args.batch, with_fallback=True)
    reps = 2000
    t0 = time.perf_counter()
    for i in range(reps):
        mlu.select(64 + i, "fp64", batch=1 + (i % 3) * 500)
    c_us = (time.perf_counter() - t0) / reps * 1e6
    sel = S.Selector()
    t0 = time.perf_counter()
    for i in range(reps):
        sel.predict(64 + i, "fp64", batch=1 + (i % 3) * 500)
    py_us = (time.perf_counter() - t0) / reps * 1e6
    report = None
    rp = os.path.join(os.path.dirname(S.MODEL_PATH), "selector_report.json")
    if os.path.exists(rp):
        with open(rp) as f:
            report = json.load(f)
    out = {"choice_for_workload": {"variant": choice[0], "nb": choice[1], "defers_to_autotuner": choice[2]},
           "choice_for_batch_of_order_256": {"batch": args.batch, "variant": choice_batched[0],
                                             "nb": choice_batched[1], "defers_to_autotuner": choice_batched[2]},
           "inference_us_c_abi": round(c_us, 2), "inference_us_python": round(py_us, 2), "training_report": report}
    log(f"selector: {out}")
    return out


def mixed_section(args, dev):
    """FP32- and BF16-product LU + FP64 refinement (mlu_dsgesv_ir) against the plain FP64
    solve (the same entry point with FP64 products and no correction: getrf,
    getrs, one residual) on A = Q diag(sv) Q^T, Q Haar, for several condition
    numbers; one right-hand side b ~ N(0, 1).  Both timed with HIP events on
    the current stream, inputs resident, the best of a few runs."""
    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    n = args.n
    log(f"mixed: Haar Q of order {n}")
    q = D.haar_orthogonal(n, seed=0, device=dev)
    b = D.gaussian_rhs(n, 1, seed=1, device=dev)
    rc, nbytes = mlu.mlu_dsgesv_ir_workspace(n, 1)
    mlu.check(rc, "mlu_dsgesv_ir_workspace")
    work_ir = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    x64 = torch.empty((n, 1), dtype=torch.float64, device=dev)
    xmp = torch.empty((n, 1), dtype=torch.float64, device=dev)
    rc, gbytes = mlu.mlu_dsgesv_gmres_ir_workspace(n, args.max_krylov)
    mlu.check(rc, "mlu_dsgesv_gmres_ir_workspace")
    work_g = torch.empty(gbytes, dtype=torch.uint8, device=dev)
    b1 = b.view(n)
    xg = torch.empty(n, dtype=torch.float64, device=dev)

    def timed(fn, reps=2):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    def berr_of(A, x):
        r = b - A @ x
        an = A.abs().sum(dim=1).max()
        return float(r.abs().max() / (an * x.abs().max() + b.abs().max()))

    cases = []
    for cond in [float(c) for c in args.mixed_conds.split(",")]:
        A = D.spectrum_matrix(q, cond)
        torch.cuda.synchronize()
        out = {}

        def fp64():   # the same solver with FP64 products and no correction: getrf + getrs + one residual
            out["r64"] = mlu.gesv_ir(A, b, precision="fp64", tol=1e-13, max_iter=0, variant=args.variant,
                                     nb=args.nb, nb_inner=args.nb_inner, X=x64, work=work_ir)

        fp64()   # warm-up
        t64 = timed(fp64)
        for low, max_iter in (("fp32", 10), ("bf16", 30)):
            if low not in args.mixed_precisions.split(","):
                continue
            def mixedrun():
                out["r"] = mlu.gesv_ir(A, b, precision=low, tol=1e-13, max_iter=max_iter, variant=args.variant,
                                       nb=args.nb, nb_inner=args.nb_inner, X=xmp, work=work_ir)

            mixedrun()   # warm-up
            tmp = timed(mixedrun)
            _, _, minfo, iters, berr = out["r"]
            ok = float(berr.item()) <= 1e-13   # a speed-up only for a solve that reached the target
            case = {"cond": cond, "precision": low, "max_iter": max_iter, "ms_fp64_solve": round(t64, 3),
                    "ms_mixed_ir": round(tmp, 3), "speedup": round(t64 / tmp, 3) if ok else None,
                    "iters": int(iters.item()),
                    "berr": float(berr.item()), "berr_fp64_solve": float(out["r64"][4].item()),
                    "berr_fp64_recomputed": berr_of(A, x64), "berr_recomputed": berr_of(A, xmp),
                    "info": int(minfo.item()),
                    "rel_diff_vs_fp64_solve": float((xmp - x64).abs().max() / x64.abs().max())}
            # LU-IR with the GMRES-IR fallback (mlu_dsgesv_gmres_ir, auto): the plain
            # corrections while they at least halve berr, GMRES corrections after
            out["g"] = None

            def gmresrun():
                out["g"] = mlu.gesv_gmres_ir(A, b1, precision=low, solver="auto", tol=1e-13, max_outer=10,
                                             max_krylov=args.max_krylov, gmres_tol=1e-6, variant=args.variant,
                                             nb=args.nb, nb_inner=args.nb_inner, x=xg, work=work_g)

            tg = timed(gmresrun, reps=1)
            _, _, ginfo, gouter, ginner, gberr = out["g"]
            case["gmres_ir_auto"] = {"ms": round(tg, 3), "speedup": round(t64 / tg, 3) if gberr <= 1e-13 else None,
                                     "outer": gouter,
                                     "inner": ginner, "berr": gberr, "berr_recomputed": berr_of(A, xg.view(n, 1)),
                                     "info": int(ginfo.item()),
                                     "rel_diff_vs_fp64_solve": float((xg.view(n, 1) - x64).abs().max()
                                                                     / x64.abs().max())}
            log(f"mixed cond={cond:g} {low}: {case}")
            cases.append(case)
        del A
    return {"what": "FP32- and BF16-product trailing updates (FP32 accumulation; FP64 panel, solves, residual, "
                    "correction) + FP64 iterative refinement to backward error <= 1e-13, vs the FP64 solve "
                    "(getrf + getrs + residual); per case LU-IR (mlu_dsgesv_ir) and LU-IR with the GMRES-IR "
                    "fallback (mlu_dsgesv_gmres_ir, auto: GMRES corrections once a plain one fails to halve berr; "
                    f"GMRES tolerance 1e-6, Krylov limit {args.max_krylov}, at most 10 corrections)",
            "n": n, "nrhs": 1, "matrix": "Q diag(logspace(0,-log10 cond,n)) Q^T, Q Haar (seed 0), b ~ N(0,1)",
            "cases": cases}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--variant", default="la", choices=["rl", "ll", "la"])
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--nb-inner", type=int, default=16)
    ap.add_argument("--inner", default="rl", choices=["rl", "ll"], help="algorithm of the panel factorization")
    ap.add_argument("--no-uniform", action="store_true", help="skip the U(0,1) (the paper's matrices) row")
    ap.add_argument("--matrix", default="spd", choices=["spd", "uniform"])
    ap.add_argument("--cpu-n", type=int, default=8192, help="size of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision + refinement measurement")
    ap.add_argument("--mixed-conds", default="1e2,1e5,1e8")
    ap.add_argument("--mixed-precisions", default="fp32,bf16", help="product precisions of the mixed rows")
    ap.add_argument("--max-krylov", type=int, default=200, help="GMRES-IR Krylov dimension limit")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-LU measurement")
    ap.add_argument("--no-et", action="store_true", help="skip the early-termination comparison")
    ap.add_argument("--no-ws", action="store_true", help="skip the worker-sharing on / off comparison")
    ap.add_argument("--no-schedule", action="store_true", help="skip the per-iteration block-size comparison")
    ap.add_argument("--lead-schedule", action="store_true",
                    help="time the main step with blocks of 2*nb over the first 3/8 of the order, then nb "
                         "(not the named workload: that one is constant nb)")
    ap.add_argument("--grid", action="store_true",
                    help="also time every variant at n in {4096, 8192, 16384} x nb in {64, 128, 256}")
    ap.add_argument("--batch", type=int, default=20000)
    ap.add_argument("--batch-host-inputs", action="store_true",
                    help="build the batched inputs on the host (B B^T in numpy, another random stream), so that "
                         "no vendor GEMM runs in the process; for counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise 1 GiB -> 1 GiB copy (reference kernel for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library factors each matrix on one GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mlu.load()
    dev = torch.device("cuda:0")
    n, K, W = args.n, args.steps, args.warmup
    flops = 2.0 * n ** 3 / 3.0

    log(f"generating {args.matrix} n={n} and {K + W + 1} resident copies")
    A = D.spd_bbt(n, seed=0, device=dev) if args.matrix == "spd" else D.uniform01(n, seed=0, device=dev)
    copies = [A.clone() for _ in range(K + W)]
    work = mlu.workspace(dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    if args.copy_calibration:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (x * 1.0)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    main_sched = lead_schedule(n, args.nb) if args.lead_schedule else None

    def step(M):
        mlu.getrf(M, variant=args.variant, nb=args.nb, nb_inner=args.nb_inner, schedule=main_sched, ipiv=ipiv,
                  info=info, work=work, inner=args.inner)

    check = {}
    for w in range(W):   # the host-side check runs after the first warm-up, so the last one leads into the timing
        step(copies[w])
        torch.cuda.synchronize()
        if w == 0:
            check = {"info": int(info.item()),
                     "sampled_residual": sampled_residual(A, copies[0], ipiv)}
            log(f"warmup 0 done: {check}")
            if W == 1:   # keep the device busy right before the timed region
                step(copies[0])
                torch.cuda.synchronize()
    if W == 0:
        log("no warmup: correctness check skipped")

    torch.cuda.synchronize()
    rc = mlu.mlu_trace_begin(4096)
    mlu.check(rc, "mlu_trace_begin")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(K):
        step(copies[W + i])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    rc, launches, gemm_ms, gemm_flops, gemm_bytes = mlu.mlu_trace_end()
    mlu.check(rc, "mlu_trace_end")
    ms_step = ms / K
    value = flops / (ms_step / 1e3) / 1e9
    log(f"timed {K} steps: {ms_step:.3f} ms/step (wall {wall / K * 1e3:.3f}), {value:.1f} GFLOP/s")
    if K > 0 and W > 0:
        check["info_last"] = int(info.item())

    roof = None
    if launches > 0:
        per_launch_flops = gemm_flops / launches
        per_launch_s = gemm_ms / launches / 1e3
        achieved = per_launch_flops / per_launch_s / 1e12
        counted = (n == 16384 and args.nb == 256 and args.variant == "la" and main_sched is None
                   and args.nb_inner == 16 and args.inner == "rl")
        rec = traffic_record() if counted else None
        traffic = None
        if rec is not None:   # per traced launch: RU2 plus the helpers that join it
            traffic = rec["fetch_bytes_per_step"] + rec["write_bytes_per_step"]
        mrec = mfma_record() if counted else None
        busy = None
        if mrec is not None and TRAFFIC_KERNEL[args.variant] in mrec.get("kernels", {}):
            busy = mrec["kernels"][TRAFFIC_KERNEL[args.variant]]["mfma_busy_frac"]
        roof = {
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "mfma_busy_frac": busy,
            "mfma_busy_note": "rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES per GRBM_GUI_ACTIVE cycle of the traced kernel "
                              "over that of a calibration kernel with every matrix unit busy, per dispatch with "
                              "dispatches serialized (profiles/mfma_counters_la_n16384.md)",
            "kernel": KERNEL_LABEL[args.variant],
            "launches": launches,
            "avg_launch_us": round(gemm_ms / launches * 1e3, 3),
            "algorithmic_flops_per_launch": per_launch_flops,
            "algorithmic_bytes_per_launch": gemm_bytes / launches,
            "share_of_step_time": round(gemm_ms / ms, 4),
        }

    sel = selector_section(args)

    uniform = None
    if not args.no_uniform and args.matrix == "spd":
        del copies
        torch.cuda.empty_cache()
        copies = None
        uniform = uniform_section(args, dev, work, ipiv, info)

    grid = grid_section(args, dev) if args.grid else None

    et = None
    if not args.no_et:
        et = et_section(args, A, ipiv, info, work)

    ws = None
    if not args.no_ws and args.variant == "la":
        ws = ws_section(args, A, ipiv, info, work)

    blocks = None
    if not args.no_schedule:
        blocks = schedule_section(args, A, ipiv, info, work)

    batched = None
    if not args.no_batched:
        batched = batched_section(args, dev)

    mixed = None
    if not args.no_mixed:
        copies = None
        torch.cuda.empty_cache()
        mixed = mixed_section(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: C oracle on n={args.cpu_n}")
        cpu = cpu_baseline(args.cpu_n)
        log(f"cpu baseline: {cpu['value']} GFLOP/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"getrf FP64 n={n} {'A=B*B^T+n*I, B~N(0,1)' if args.matrix == 'spd' else 'U(0,1)'} "
                        f"(seed 0), variant={args.variant.upper()}, nb={args.nb}, nb_inner={args.nb_inner}"
                        + (", inner=LL" if args.inner == "ll" else "")
                        + (f", first {len(main_sched)} blocks of {main_sched[0]}" if main_sched else ""),
            "n": n,
            "variant": args.variant,
            "nb": args.nb,
            "nb_inner": args.nb_inner,
            "inner": args.inner,
            "schedule": main_sched,
            "matrix": args.matrix,
            "parallelism": "single GPU",
        },
        "frac_fp64_peak": round(value / (FP64_PEAK_TFLOPS * 1e3), 4),
        "roofline": roof,
        "uniform01": uniform,
        "mixed": mixed,
        "early_termination": et,
        "worker_sharing": ws,
        "block_schedule": blocks,
        "selector": sel,
        "grid": grid,
        "batched": batched,
        "cpu_baseline": cpu,
        "check": check,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
