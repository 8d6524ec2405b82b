"""Builds libglint.so (HIP for gfx950) in-tree.

    python -m paper_2306_05051_amd.build

hipcc compiles every HIP translation unit for gfx950 only, with packed FP32
instructions disabled (-packed-fp32-ops), then links one shared library next
to this file.  Object files go to _build/ (not committed).  It also builds
valu_probe, the stand-alone VALU issue-rate probe behind the roofline's
denominator and slot costs (costmodel.py).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libglint.so")
PROBE = os.path.join(HERE, "valu_probe")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["glint_fwd.hip", "glint_order.hip", "glint_bwd.hip"]
# Per-source flags.  The adjoint's work-unit kernel loops over the chunks of
# lit pixels it covers and redoes a chunk's pixel set-up inside that loop;
# machine loop-invariant code motion hoisted the set-up's FP64 constants to
# the kernel entry, where they spilled to scratch (about 0.85 GB of scratch
# traffic per 4K adjoint call).  Without it the kernel fits in 128 VGPRs
# with no spill and runs 19% faster; the forward keeps the pass (it is 3%
# slower without it).  Scheduling: the forward's occupancy is fixed at 4
# waves per SIMD by its LDS, so the scheduler that favours instruction-level
# parallelism over registers (116 VGPRs instead of 106, no spill) is 0.8%
# faster on the 4K frame; the adjoint gains 2.7% from the iterative ILP
# scheduler (same-box alternations of the two builds).
SOURCE_FLAGS = {
    "glint_fwd.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "glint_bwd.hip": ["-mllvm", "-disable-machine-licm", "-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libglint.so failed")
    os.replace(tmp, OUT)
    r = subprocess.run([HIPCC, *FLAGS, "-o", PROBE + ".tmp", os.path.join(CSRC, "valu_probe.hip")],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on valu_probe.hip")
    os.replace(PROBE + ".tmp", PROBE)
    if verbose:
        print("built", OUT, "and", PROBE)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
