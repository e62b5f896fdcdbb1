"""Build libmlu.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmlu.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


CALIB_SRC = os.path.join(HERE, "calib", "mfma_peak.hip")
CALIB_BIN = os.path.join(HERE, "calib", "mfma_peak")


def build_calibration(verbose: bool = False) -> str:
    """The matrix-core calibration program used by the counter profiles."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    tmp = CALIB_BIN + ".tmp"
    cmd = ["hipcc", *flags, "-o", tmp, CALIB_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building the calibration program")
    os.replace(tmp, CALIB_BIN)
    return CALIB_BIN


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmlu.so")
    os.replace(tmp, LIB)
    return LIB


PROBE_LIB = os.path.join(HERE, "libmlu_probe.so")


def build_probe(verbose: bool = False) -> str:
    """libmlu_probe.so: the same sources with the panel kernel's exact-mode
    column stamps compiled in (MLU_PANEL_PROBE), for probe_panel.py; never
    loaded by the library's users."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = PROBE_LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-DMLU_PANEL_PROBE", "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmlu_probe.so")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build_all(verbose: bool = False) -> list[str]:
    """libmlu.so and libmlu_probe.so, compiled side by side (two hipcc
    processes), then the calibration program."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = []
    for out, extra in ((LIB, []), (PROBE_LIB, ["-DMLU_PANEL_PROBE"])):
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-o", out + ".tmp", *srcs]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for out, proc in jobs:
        log, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(log)
            failed.append(os.path.basename(out))
        else:
            os.replace(out + ".tmp", out)
    if failed:
        raise RuntimeError("hipcc failed building " + ", ".join(failed))
    return [LIB, PROBE_LIB, build_calibration(verbose)]


if __name__ == "__main__":
    for path in build_all(verbose=True):
        print(path)
