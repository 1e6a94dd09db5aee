"""Build libmifft.so (HIP, gfx950) in-tree with hipcc.

Every kernel translation unit is compiled for gfx950 only; the FP32 Stockham
file is compiled once per transform length (-DMIFFT_LOG2N=1..14), the
real-input file once per half length (-DMIFFT_LOG2M=0..14).  Objects go
to ``_build/`` beside this file, the library to ``libmifft.so`` beside it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmifft.so")
# measurement support for the benchmark: a plain streaming copy (HBM ceiling)
COPY_LIB = os.path.join(HERE, "libstreamcopy.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for every device compile.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
                "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _units():
    units = []
    for L in range(1, 15):
        units.append(("fft_c32.hip", f"fft_c32_L{L}.o", [f"-DMIFFT_LOG2N={L}"]))
    for L in range(1, 12):
        units.append(("fused_loss.hip", f"fused_loss_L{L}.o", [f"-DMIFFT_LOG2N={L}"]))
    for L in range(0, 15):
        units.append(("real.hip", f"real_M{L}.o", [f"-DMIFFT_LOG2M={L}"]))
    units.append(("twiddle.hip", "twiddle.o", []))
    units.append(("fourstep.hip", "fourstep.o", []))
    units.append(("nd.hip", "nd.o", []))
    units.append(("nd2.hip", "nd2.o", []))
    units.append(("nd3.hip", "nd3.o", []))
    for wg in (64, 128, 256):
        units.append(("ragged.hip", f"ragged_wg{wg}.o", [f"-DMIFFT_RAGGED_WG={wg}"]))
    units.append(("ragged_plan.cpp", "ragged_plan.o", ["-x", "hip"]))
    units.append(("half.hip", "half.o", []))
    for L in range(1, 11):
        units.append(("half_small.hip", f"half_small_L{L}.o", [f"-DMIFFT_LOG2N={L}"]))
    units.append(("api.cpp", "api.o", ["-x", "hip"]))
    return units


def _compile(src, obj, extra):
    cmd = [HIPCC] + DEVICE_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {extra}:\n{r.stderr}")
    return r.stderr


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(16, max(1, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, *u) for u in units]
        for f in futs:
            msg = f.result()
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    objs = [os.path.join(BUILD, u[1]) for u in units]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    _compile("stream_copy.hip", "stream_copy.o", [])
    tmp = COPY_LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
                        os.path.join(BUILD, "stream_copy.o")], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of the copy library failed:\n{r.stderr}")
    os.replace(tmp, COPY_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
