"""Writes oracle_regression.json: digests of the CPU oracle's outputs on small seeded cases.

These are regression fixtures of the oracle itself, not pins of the model: the pins are the closed forms,
library routines and invariants in tests/test_oracle_*.py. A digest that changes means the oracle's
arithmetic changed; such a change must name, in its commit message, the passage of the paper (or the
reading of it) that justifies it, and this script is then re-run. Calls only the oracle and the seeded
input generators.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.json")


def digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.dtype.str.encode() + str(a.shape).encode() + a.tobytes()).hexdigest()[:32]


def cases() -> dict:
    out = {}
    w = synth.make_workload("tiny")
    nrm = oracle.normals(w.dem, w.cell_size)
    mask = oracle.release_mask(nrm, w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    out["tiny_normals"] = digest(nrm)
    out["tiny_mask"] = digest(mask)
    r = oracle.trajectories(w.dem, mask, w.cell_size, oracle.make_params(**w.params), 4, 500, w.seed)
    out["tiny_p4_s500"] = {"counts": digest(r.counts), "vmax": digest(r.vmax),
                           "stats": [r.steps, r.n_exit, r.n_stop, r.n_limit]}
    r64 = oracle.trajectories(w.dem, mask, w.cell_size, oracle.make_params(**w.params), 1, 300, w.seed, prec="f64")
    out["tiny_p1_s300_f64"] = {"counts": digest(r64.counts), "vmax": digest(r64.vmax),
                               "stats": [r64.steps, r64.n_exit, r64.n_stop, r64.n_limit]}
    fine = oracle.release_mask_fine(nrm, w.dem, 3, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    sub = np.zeros_like(fine)
    sub[::5, ::5] = fine[::5, ::5]
    rf = oracle.trajectories_fine(w.dem, sub, 3, w.cell_size, oracle.make_params(**w.params), 2, 300, w.seed)
    out["tiny_fine3"] = {"mask": digest(fine), "counts": digest(rf.counts), "vmax": digest(rf.vmax),
                         "stats": [rf.steps, rf.n_exit, rf.n_stop, rf.n_limit]}
    out["tiny_snow"] = digest(oracle.snow_cover(nrm, w.dem, float(np.median(w.dem)), 100.0, 40.0, 8.0))
    levels = oracle.mipmap(r.counts, r.vmax)
    out["tiny_mipmap"] = {"counts": [digest(c) for c, _ in levels], "vmax": [digest(v) for _, v in levels]}
    p = oracle.make_params(mu=0.25, xi=1500.0)
    small = np.zeros_like(mask)
    small[::4, ::4] = mask[::4, ::4]
    sf = oracle.smooth_forward(w.dem, small, w.cell_size, p, 4, 500, w.seed)
    out["tiny_smooth"] = {"dep_q": digest(sf.dep_q), "stats": [sf.steps, sf.n_exit, sf.n_stop, sf.n_limit]}
    gD = (np.random.default_rng(3).random(w.dem.shape) - 0.5).astype(np.float32)
    g = oracle.smooth_backward(w.dem, small, w.cell_size, p, 4, 500, w.seed, gD)
    out["tiny_adjoint"] = {"dmu": g.dmu, "dxi": g.dxi, "dh": g.dh, "dmass": digest(g.dmass)}
    return out


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(cases(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", OUT)
