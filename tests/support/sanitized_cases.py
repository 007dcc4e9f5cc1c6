"""Oracle calls exercised by the host sanitizer test: every C entry point of the oracle, on small seeded
inputs whose particles end in every way (grid exit, energy stop, runout-angle stop, step limit). `run()`
returns the outputs as a flat dict of arrays, so the sanitised build and the normal build can be compared
bit for bit."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def _inputs():
    dem = synth.alpine_dem(64, 500.0, seed=21)[:41, :57].copy()
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 25.0, 50.0, float(np.quantile(dem, 0.5)), np.inf)
    mass = np.random.default_rng(3).uniform(0.5, 1.5, dem.shape).astype(np.float32)
    gD = np.random.default_rng(4).standard_normal(dem.shape).astype(np.float32)
    return dem, nrm, mask, mass, gD


def run() -> dict:
    dem, nrm, mask, mass, gD = _inputs()
    out = {"philox": oracle.philox([1, 2, 3, 4], [5, 6]), "normals": nrm, "mask": mask,
           "cells": oracle.compact(mask), "snow": oracle.snow_cover(nrm, dem, 250.0, 40.0, 40.0, 6.0)}
    fine = oracle.release_mask_fine(nrm, dem, 3, 25.0, 50.0, float(np.quantile(dem, 0.5)), np.inf)
    out["mask_fine"] = fine
    cases = {"drag": dict(mu=0.12, xi=1500.0), "angle": dict(mu=0.05, xi=2500.0, tan_alpha=0.45),
             "limit": dict(mu=0.01, xi=np.inf, randomness=0.1)}
    for name, kw in cases.items():
        p = oracle.make_params(**kw)
        S = 25 if name == "limit" else 400
        for prec in ("f32", "f64"):
            r = oracle.trajectories(dem, mask, 10.0, p, 3, S, 7, 1, prec=prec)
            out[f"traj_{name}_{prec}"] = np.concatenate([r.counts.ravel().astype(np.float64), r.vmax.ravel(),
                                                         [r.steps, r.n_exit, r.n_stop, r.n_limit]])
            sm = oracle.smooth_forward(dem, mask, 10.0, p, 3, S, 7, 1, mass=mass, vel_splat=True, prec=prec)
            out[f"smooth_{name}_{prec}"] = np.concatenate([sm.dep_q.ravel(), sm.vel_q.ravel()])
            g = oracle.smooth_backward(dem, mask, 10.0, p, 3, S, 7, gD, 1, mass=mass, prec=prec)
            out[f"grad_{name}_{prec}"] = np.concatenate([[g.dmu, g.dxi, g.dh], g.dmass.ravel(),
                                                         g.per_particle.ravel().astype(np.float64)])
            Lp, reason, steps = oracle.smooth_particles(dem, mask, 10.0, p, 3, S, 7, gD, 1, mass=mass, prec=prec)
            out[f"particles_{name}_{prec}"] = np.concatenate([Lp, reason, steps])
        out[f"tangent_{name}"] = np.asarray(oracle.smooth_tangent(dem, mask, 10.0, p, 3, S, 7, gD, 1, mass=mass))
        rf = oracle.trajectories_fine(dem, fine, 3, 10.0, p, 2, S, 7, 1)
        out[f"fine_{name}"] = np.concatenate([rf.counts.ravel().astype(np.float64), rf.vmax.ravel()])
        tr = oracle.trace(dem, 10.0, p, 20, 30, 1, S, 7, 1)
        out[f"trace_{name}"] = tr.rows.ravel()
        levels = oracle.mipmap(r.counts, r.vmax.astype(np.float32))
        out[f"mip_{name}"] = np.concatenate([np.concatenate([c.ravel().astype(np.float64), v.ravel()])
                                             for c, v in levels])
    return out


if __name__ == "__main__":
    import sys
    np.savez(sys.argv[1], **run())
