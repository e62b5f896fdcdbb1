"""Per-column phase times of the panel kernel's exact-mode column step.

Loads libmlu_probe.so (the library built with the kernel's real-time stamps,
MLU_PANEL_PROBE; see build.py), factors U(0, 1) m x 16 blocks with
mlu_dgetf2_block (pivoting at nearly every column, so the block runs in exact
mode after the speculative attempt), and prints, for the first and the last
workgroup, the mean time of each phase of the 16 column steps:

  local_best  the local argmax, its barrier and the reduction over the waves
  to poll     from there to the first poll of the other workers' candidates
  poll        the poll itself (the other workers' candidates through memory)
  sync        the barrier that hands the winner to every thread
  apply       the interchange, division and row update

python -m paper_1611_06365_amd.probe_panel [--m 16384 8192 4096] [--reps 3]
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TICK_US = 0.01   # s_memrealtime counts at 100 MHz
PHASES = ("local_best", "to poll", "poll", "sync", "apply")


def main(argv=None) -> int:
    import numpy as np
    import torch

    import inputs as G
    from paper_1611_06365_amd import build, mlu

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--m", type=int, nargs="+", default=[16384, 8192, 4096])
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    if not os.path.exists(build.PROBE_LIB):
        raise SystemExit(f"{build.PROBE_LIB} is missing: python -m paper_1611_06365_amd.build")
    mlu.load(build.PROBE_LIB)
    raw = ctypes.CDLL(build.PROBE_LIB)
    raw.mlu_probe_stamps.argtypes = [ctypes.POINTER(ctypes.c_ulonglong)]
    for m in args.m:
        A = torch.from_numpy(G.uniform01(m, 16, seed=3)).to("cuda:0")
        for _ in range(args.reps):   # the stamps are those of the last call
            F = A.clone()
            mlu.getf2_block(F)
            torch.cuda.synchronize()
        buf = (ctypes.c_ulonglong * (2 * 64 * 6))()
        if raw.mlu_probe_stamps(buf) != 0:
            raise SystemExit("mlu_probe_stamps failed")
        t = np.array(buf, dtype=np.float64).reshape(2, 64, 6)
        for who, name in ((0, "first"), (1, "last")):
            d = np.diff(t[who, :16, :], axis=1) * TICK_US
            period = (t[who, 1:16, 0] - t[who, :15, 0]) * TICK_US
            parts = ", ".join(f"{p} {d[:, i].mean():.2f}" for i, p in enumerate(PHASES))
            print(f"m={m} {name} worker: per column us: {parts}; column period {period.mean():.2f}", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
