"""Build the CPU oracle twins: liboracle_f32.so and liboracle_f64.so (plain gcc, no FMA contraction).

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> None:
    src = os.path.join(_HERE, "avl_oracle.c")
    for prec, extra in (("f32", []), ("f64", ["-DAVL_F64"])):
        out = os.path.join(_HERE, f"liboracle_{prec}.so")
        tmp = out + ".tmp"
        cmd = ["gcc", *FLAGS, *extra, src, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


# Host sanitizer build (tests only): AddressSanitizer and UndefinedBehaviorSanitizer (float-to-int
# overflow included, every report fatal), with every uninitialised local filled with a NaN pattern so
# that a value read before it is written shows up in the results. The arithmetic flags are the same.
SAN_FLAGS = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             "-ftrivial-auto-var-init=pattern"]
SAN_CC = "/opt/rocm/llvm/bin/clang"


def asan_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that a sanitised library loaded by Python needs preloaded."""
    out = subprocess.run([SAN_CC, "-print-file-name=libclang_rt.asan-x86_64.so"], check=True, capture_output=True,
                         text=True).stdout.strip()
    return out


def build_sanitized(outdir: str) -> None:
    src = os.path.join(_HERE, "avl_oracle.c")
    for prec, extra in (("f32", []), ("f64", ["-DAVL_F64"])):
        out = os.path.join(outdir, f"liboracle_{prec}.so")
        subprocess.run([SAN_CC, *SAN_FLAGS, *extra, src, "-o", out, "-lm"], check=True)


if __name__ == "__main__":
    build(verbose=True)
