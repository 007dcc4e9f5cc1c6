"""rocRAND's Philox4x32-10 as an independent reference (host program built with hipcc on first use)."""
from __future__ import annotations

import hashlib
import os
import subprocess
import tempfile

import numpy as np

_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rocrand_philox_ref.cpp")


def _binary() -> str:
    with open(_SRC, "rb") as f:
        tag = hashlib.sha1(f.read()).hexdigest()[:12]
    out = os.path.join(tempfile.gettempdir(), f"avl_rocrand_philox_ref_{tag}")
    if not os.path.exists(out):
        tmp = out + f".{os.getpid()}"
        subprocess.run(["hipcc", "-O1", _SRC, "-o", tmp], check=True, capture_output=True)
        os.replace(tmp, out)
    return out


def philox_blocks(ctr_key: np.ndarray) -> np.ndarray:
    """ctr_key: (n, 6) uint32 rows (c0, c1, c2, c3, k0, k1) -> (n, 4) uint32 output words."""
    ctr_key = np.asarray(ctr_key, dtype=np.uint32).reshape(-1, 6)
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in ctr_key) + "\n"
    res = subprocess.run([_binary()], input=text, capture_output=True, text=True, check=True)
    out = np.array([[int(t) for t in line.split()] for line in res.stdout.strip().splitlines()], dtype=np.uint64)
    return out.astype(np.uint32).reshape(-1, 4)
