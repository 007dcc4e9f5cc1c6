#!/usr/bin/env python3
"""Benchmark of the avalanche-overlay hot path on one MI355X.

One step = one pass of the whole path over the alpine tile (2048^2 ridged fBm DEM at 10 m, ~1e5
release cells, 256 particles per cell, step limit 4000): normals -> release map -> release-cell list
-> particle trajectories -> raster finalize, with the DEM already resident in HBM. The metric is
particle-steps per second (every step a particle enters counts once).

Prints one JSON line. Extra fields: the roofline of the dominant kernel (the trajectory kernel), the
CPU oracle timed on a bounded sample of the same workload, and per-stage timings.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one particle-step of the model, counted from its definition (one op per
# add/sub/mul/div/sqrt/floor/compare/convert and per 32-bit integer mul/mulhi/xor/add/shift/clamp):
# half a Philox4x32-10 block (50), the two uniforms (10), the direction blend (24), the move and grid
# test (10), the bilinear sample with index clamps (25), the energy step (11), the cell bookkeeping (3).
OPS_PER_STEP = 133
# Vector ALU peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 VALU
# instruction per SIMD every 4 cycles) = 39.3e12 lane-ops/s; the 157.3 TFLOP/s fp32 figure counts an
# FMA as 2 and packed issue as 2.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# DEM gather (2x2 texels, 16 B) and the two 4-byte atomics per step; HBM3E peak 8 TB/s
BYTES_PER_STEP = 24
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="alpine", choices=["tiny", "alpine", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=0, help="oracle sample: every n-th release cell (0 = auto)")
    ap.add_argument("--no-batched", action="store_true", help="skip the ensemble (batched vs plain) leg")
    return ap.parse_args()


def cpu_baseline(w, mask: np.ndarray, stride: int) -> dict:
    import oracle
    cells = np.flatnonzero(mask)
    if stride <= 0:
        stride = max(1, len(cells) // 1500)
    sample = np.zeros(mask.size, np.uint8)
    sample[cells[::stride]] = 1
    sample = sample.reshape(mask.shape)
    p = oracle.make_params(**w.params)
    t0 = time.perf_counter()
    res = oracle.trajectories(w.dem, sample, w.cell_size, p, w.particles_per_cell, w.step_limit, w.seed)
    dt = time.perf_counter() - t0
    return {"value": res.steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"every {stride}th release cell ({int(sample.sum())} cells x {w.particles_per_cell} "
                      f"particles, {res.steps} particle-steps, {dt:.1f} s, single-threaded FP32 C oracle)"}


def batched_leg(avl, torch, reps: int) -> dict:
    """Ensemble sweep: 16 ridged-fBm tiles of 1024^2 at 10 m, one release scenario each (103-26,397
    cells), crossed with 64 (mu, xi, h) sets: 1024 runs of 32 particles per cell and 2000 steps. Timed
    as one batched call (captured once into a HIP graph, then replayed) and as 1024 plain calls."""
    import synth
    e = synth.make_ensemble()
    dev = torch.device("cuda", 0)
    dems = torch.from_numpy(e.dems).to(dev)
    masks = torch.from_numpy(e.masks).to(dev)
    ptab = avl.params_tensor(e.params, dev)
    rtab = avl.runs_tensor(e.runs, dev)
    stream = torch.cuda.Stream()
    out = None
    with torch.cuda.stream(stream):
        for _ in range(2):  # tune, capture, replay once
            out = avl.trajectories_batched(dems, masks, e.cell_size, ptab, rtab, e.particles_per_cell, e.step_limit, out)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = avl.trajectories_batched(dems, masks, e.cell_size, ptab, rtab, e.particles_per_cell, e.step_limit, out)
        stream.synchronize()
        t_batch = (time.perf_counter() - t0) / reps
    steps = int(out.stats.cpu().numpy()[:, 0].sum())
    variant = avl.last_variant()
    # the same runs as plain calls, each into its own slice of the output rasters
    plain = avl.BatchResult(torch.empty_like(out.counts), torch.empty_like(out.vmax), torch.empty_like(out.stats),
                            out.status)
    params = [avl.Params.make(**p) for p in e.params]

    def plain_loop():
        for k, (t, sc, p, run_id, seed) in enumerate(e.runs):
            avl.trajectories(dems[t], masks[sc], e.cell_size, params[p], e.particles_per_cell, e.step_limit, seed,
                             run_id, avl.RunResult(plain.counts[k], plain.vmax[k], plain.stats[k]))
    plain_loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain_loop()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    same = bool(torch.equal(plain.counts.view(torch.int32), out.counts.view(torch.int32))
                and torch.equal(plain.vmax, out.vmax)
                and torch.equal(plain.stats.view(torch.int64), out.stats.view(torch.int64)))
    return {"workload": "16 tiles x 64 parameter sets = 1024 runs, 1024^2 at 10 m, 32 particles/cell, "
                        "2000 steps, scenarios 103-26397 cells",
            "runs": len(e.runs), "particles": int(e.masks.sum(axis=(1, 2))[[r[1] for r in e.runs]].sum()
                                                   * e.particles_per_cell),
            "particle_steps": steps, "ms_batched": t_batch * 1e3, "ms_plain_calls": t_plain * 1e3,
            "speedup_batched_vs_plain": t_plain / t_batch,
            "particle_steps_per_s_batched": steps / t_batch, "particle_steps_per_s_plain": steps / t_plain,
            "variant": variant, "batched_equals_plain": same}


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "detail": "particles are independent; a multi-GPU run would split particle ranges and "
                                    "all-reduce the integer rasters (see the design notes)"}))
        return 2
    import torch
    import synth
    import paper_2506_23364_amd as avl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    torch.cuda.set_device(0)
    w = synth.make_workload(args.workload)
    h, wd = w.dem.shape
    dem = torch.from_numpy(w.dem).cuda()
    params = avl.Params.make(**w.params)
    stream = torch.cuda.current_stream()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    res = None

    def step(timed: bool):
        nonlocal res
        if timed:
            ev[0].record(stream)
        nrm = avl.normals(dem, w.cell_size)
        mask = avl.release_mask(nrm, dem, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
        if timed:
            ev[1].record(stream)
        res = avl.trajectories(dem, mask, w.cell_size, params, w.particles_per_cell, w.step_limit, w.seed, 0, res)
        if timed:
            ev[2].record(stream)
        return mask

    for _ in range(max(args.warmup, 1)):
        mask = step(False)
    torch.cuda.synchronize()
    stats = res.stats.cpu().numpy().astype(np.int64)
    steps_per_pass = int(stats[0])
    n_release = int(mask.sum().item())
    mask_np = mask.cpu().numpy()

    t_terrain = t_traj = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        ev[2].synchronize()
        t_terrain += ev[0].elapsed_time(ev[1])
        t_traj += ev[1].elapsed_time(ev[2])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # a second loop without per-step syncs gives the throughput figure
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert int(res.stats.cpu().numpy()[0]) == steps_per_pass, "particle-step count changed between passes"

    value = steps_per_pass * args.steps / elapsed
    traj_s = t_traj / 1e3 / args.steps
    achieved_tops = OPS_PER_STEP * steps_per_pass / traj_s / 1e12
    out = {
        "metric": "particle-steps/s forward + s per (mu,xi) gradient, batched vs plain, 1 MI355X",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {h}x{wd} ridged diamond-square fBm DEM at {w.cell_size:g} m, release "
                        f"{w.slope_min_deg:g}-{w.slope_max_deg:g} deg above z={w.z_min:.1f} m "
                        f"({n_release} cells), {w.particles_per_cell} particles/cell, step limit {w.step_limit}, "
                        f"mu {w.params['mu']:g}, xi {w.params['xi']:g}, h {w.params['flow_height']:g}, "
                        f"persistence {w.params['persistence']:g}, randomness {w.params['randomness']:g}",
            "release_cells": n_release,
            "particles": n_release * w.particles_per_cell,
            "particle_steps_per_pass": steps_per_pass,
            "mean_steps_per_particle": steps_per_pass / max(1, n_release * w.particles_per_cell),
            "ends_exit_stop_limit": [int(v) for v in stats[1:]],
        },
        "timing": {
            "ms_terrain_normals_mask": t_terrain / args.steps,
            "ms_trajectories_call": t_traj / args.steps,
            "ms_per_step_synced": wall / args.steps * 1e3,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_trajectories",
            "achieved": achieved_tops,
            "peak": ALU_PEAK_TOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tops / ALU_PEAK_TOPS,
            "traffic": None,
            "ops_per_particle_step": OPS_PER_STEP,
            "hbm_view": {"bytes_per_particle_step": BYTES_PER_STEP,
                         "achieved_GBs": BYTES_PER_STEP * steps_per_pass / traj_s / 1e9,
                         "peak_GBs": HBM_PEAK_GBS},
        },
    }
    if not args.no_batched:
        out["batched"] = batched_leg(avl, torch, 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, mask_np, args.cpu_stride)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
