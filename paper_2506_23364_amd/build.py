"""Build libavl.so (the HIP library behind include/avl.h) in-tree for gfx950.

Flags that the bit-exact contract depends on: no FP contraction, IEEE binary32 division and square
root correctly rounded, denormals kept, no packed-FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/api.hip", "csrc/terrain.hip", "csrc/trajectories.hip", "csrc/smooth.hip", "csrc/membench.hip"]
LIB = os.path.join(HERE, "libavl.so")
ARCH = os.environ.get("AVL_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the kernels' same-address atomics on hot paths are issued by one lane already (queue and budget
    # counters, statistics); the compiler's wave-level combining only adds lane counting around them
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *HIP_FLAGS, *(extra or []), f"-I{os.path.join(ROOT, 'include')}", *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libavl.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
