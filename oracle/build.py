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


if __name__ == "__main__":
    build(verbose=True)
