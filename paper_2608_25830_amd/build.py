"""Build libgtmp.so (HIP for gfx950) in-tree.

    python -m paper_2608_25830_amd.build [--asm]

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, and linked into one shared library next to this file.
``--asm`` also writes the device assembly of each source under ``_build/``
for inspection.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgtmp.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]

SOURCES = ["api.hip", "sample.hip", "edge.hip", "sweep.hip", "anytime.hip", "batch.hip", "surrogate.hip",
           "classes.hip", "simplify.hip", "rrtc.hip", "lazy.hip", "select.hip"]
# the growing-budget sampler and its pair ranking, the class labels and the
# RRT-Connect decisions are defined as FP32 computations with a fixed
# operation order: no contraction into fused multiply-adds in those files
EXTRA = {src: ["-ffp-contract=off"] for src in ("anytime.hip", "classes.hip", "rrtc.hip", "select.hip")}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _asm(src: str) -> None:
    out = os.path.join(BUILD, os.path.splitext(src)[0] + f"-{ARCH}.s")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)


def build(asm: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
        if asm:
            list(ex.map(_asm, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(asm="--asm" in sys.argv))
