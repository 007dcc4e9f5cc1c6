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
# HBM traffic of the trajectory kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, recorded with the
# hash of the kernel sources it was measured on; reported only while the sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_trajectories_alpine_traffic.md")
KERNEL_SOURCES = ["paper_2506_23364_amd/csrc/trajectories.hip", "paper_2506_23364_amd/csrc/particle.h",
                  "paper_2506_23364_amd/csrc/avl_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(variant: int):
    """Memory-side bytes per launch of kernel variant `variant` from the committed counter summary, or
    None when the summary has no figure for it or was taken on other kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch[") or line.startswith("source_sha256:"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    key = f"traffic_bytes_per_launch[{variant}]"
    if key not in vals or vals.get("source_sha256") != kernel_source_hash():
        return None
    return float(vals[key])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="alpine", choices=["tiny", "alpine", "large"])
    ap.add_argument("--variant", type=int, default=-1,
                    help="trajectory kernel variant (default -1: the library's autotuner chooses)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes of the full-pass oracle run (0 to skip it)")
    ap.add_argument("--cpu-stride", type=int, default=0, help="oracle sample: every n-th release cell (0 = auto)")
    ap.add_argument("--no-batched", action="store_true", help="skip the ensemble (batched vs plain) leg")
    ap.add_argument("--no-gradient", action="store_true", help="skip the calibration-gradient and calibration legs")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed passes: no mipmap, snow, fine-release, ensemble, gradient or CPU legs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 256 MiB once first: a plain copy of known size that calibrates HBM byte counters")
    return ap.parse_args()


def cpu_baseline(w, mask: np.ndarray, stride: int) -> dict:
    """The FP32 oracle, single-threaded, on every `stride`-th release cell of the workload."""
    import oracle
    cells = np.flatnonzero(mask)
    if stride <= 0:
        stride = 2
    sample = np.zeros(mask.size, np.uint8)
    sample[cells[::stride]] = 1
    sample = sample.reshape(mask.shape)
    p = oracle.make_params(**w.params)
    t0 = time.perf_counter()
    res = oracle.trajectories(w.dem, sample, w.cell_size, p, w.particles_per_cell, w.step_limit, w.seed)
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": res.steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle", "cpu": model,
            "sample": f"1 in {stride} release cells ({int(sample.sum())} cells x {w.particles_per_cell} "
                      f"particles, {res.steps} particle-steps, {dt:.1f} s, single-threaded FP32 C oracle)"}


def _oracle_part(args):
    """One worker of the parallel oracle pass: the particles of a contiguous range of release cells."""
    dem, mask_part, cell_size, params, P, S, seed = args
    import oracle
    r = oracle.trajectories(dem, mask_part, cell_size, oracle.make_params(**params), P, S, seed)
    return r.counts, r.vmax, (r.steps, r.n_exit, r.n_stop, r.n_limit)


def cpu_parallel(w, mask: np.ndarray, procs: int, gpu_counts: np.ndarray, gpu_vmax: np.ndarray) -> dict:
    """The whole pass on the oracle, run as `procs` processes over disjoint ranges of release cells and
    merged exactly (counts add, speeds take the maximum): a full-size CPU time and a full-size check of the
    GPU rasters."""
    import multiprocessing as mp
    cells = np.flatnonzero(mask)
    parts = []
    for chunk in np.array_split(cells, procs):
        m = np.zeros(mask.size, np.uint8)
        m[chunk] = 1
        parts.append((w.dem, m.reshape(mask.shape), w.cell_size, w.params, w.particles_per_cell, w.step_limit,
                      w.seed))
    ctx = mp.get_context("spawn")  # fresh interpreters: the children never touch the GPU
    with ctx.Pool(procs) as pool:
        pool.map(_oracle_part, parts[:1])  # start-up and library load, untimed
        t0 = time.perf_counter()
        out = pool.map(_oracle_part, parts)
        dt = time.perf_counter() - t0
    counts = np.sum([o[0] for o in out], axis=0, dtype=np.uint64).astype(np.uint32)
    vmax = np.max([o[1] for o in out], axis=0)
    steps = sum(o[2][0] for o in out)
    same = bool(np.array_equal(counts, gpu_counts) and np.array_equal(vmax, gpu_vmax))
    return {"value": steps / dt, "unit": "particle-steps/s", "processes": procs, "seconds": dt,
            "particle_steps": int(steps), "gpu_rasters_equal_oracle": same}


def mipmap_leg(avl, torch, res, reps: int) -> dict:
    """The multi-resolution overlay of the pass's rasters: every coarser level of counts and speeds.
    Timed as replays of a captured HIP graph of the call (two kernel launches), so host overhead is out."""
    h, w = res.counts.shape
    n = h * w
    levels = int(avl.lib.avl_mipmap_levels(h, w))
    cells = int(avl.lib.avl_mipmap_cells(h, w))
    cp = torch.empty(cells, dtype=torch.uint64, device="cuda")
    vp = torch.empty(cells, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()

    def call():
        rc = avl.lib.avl_overlay_mipmap(res.counts.data_ptr(), res.vmax.data_ptr(), h, w, cp.data_ptr(), vp.data_ptr(),
                                        stream.cuda_stream)
        assert rc == 0, rc

    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        call()
        stream.synchronize()
        eager = vp.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            call()
        g.replay()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 8 * n + 12 * cells  # read level 0 (u32 + f32), write every coarser level (u64 + f32)
    return {"levels": levels, "ms": ms, "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / ms / 1e6,
            "peak_GBs": HBM_PEAK_GBS, "replay_equals_eager": bool(torch.equal(eager, vp))}


def fine_leg(avl, torch, w, dem, reps: int, mult: int = 2, per_texel: int = 64) -> dict:
    """The same tile and release rule evaluated on a release texture with mult x mult texels per DEM cell,
    with per_texel particles per release texel (mult^2 * per_texel = the plain pass's particles per cell):
    the fine release map and the trajectory pass from it."""
    params = avl.Params.make(**w.params)
    nrm = avl.normals(dem, w.cell_size)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    mask = avl.release_mask_fine(nrm, dem, mult, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    res = avl.trajectories_fine(dem, mask, mult, w.cell_size, params, per_texel, w.step_limit, w.seed)
    torch.cuda.synchronize()
    map_ms, kern_ms = [], []
    avl.set_profiling(True)
    for _ in range(reps):
        e[0].record(stream)
        mask = avl.release_mask_fine(nrm, dem, mult, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
        e[1].record(stream)
        res = avl.trajectories_fine(dem, mask, mult, w.cell_size, params, per_texel, w.step_limit, w.seed, 0, res)
        torch.cuda.synchronize()
        map_ms.append(e[0].elapsed_time(e[1]))
        kern_ms.append(avl.last_kernel_ms())
    avl.set_profiling(False)
    texels = int(mask.count_nonzero().item())
    steps = int(res.stats[0].item())
    h, wd = dem.shape
    fine_cells = h * wd * mult * mult
    map_bytes = 20 * h * wd + fine_cells  # normals and heights once, one byte per release texel
    kms = float(np.mean(kern_ms))
    return {"mult": mult, "particles_per_texel": per_texel, "release_texels": texels,
            "particles": texels * per_texel, "particle_steps_per_pass": steps,
            "ms_release_map": float(np.mean(map_ms)), "release_map_GBs": map_bytes / float(np.mean(map_ms)) / 1e6,
            "ms_trajectory_kernel": kms, "particle_steps_per_s": steps / (kms * 1e-3)}


def snow_leg(avl, torch, w, dem, reps: int) -> dict:
    """Snow-cover alpha of the tile (section 5.1) from its normals: an HBM stream of 24 bytes per texel."""
    nrm = avl.normals(dem, w.cell_size)
    line = float(torch.quantile(dem.flatten()[::16], 0.6).item())
    stream = torch.cuda.current_stream()
    out = avl.snow_cover(nrm, dem, line, 200.0, 40.0, 8.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        out = avl.snow_cover(nrm, dem, line, 200.0, 40.0, 8.0)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 24 * dem.numel()
    return {"ms": ms, "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / ms / 1e6, "peak_GBs": HBM_PEAK_GBS,
            "covered_fraction": float((out > 0).float().mean().item()),
            "note": "per call, launch included (one kernel)"}


def calibration_leg(avl, torch, iters: int = 60) -> dict:
    """Calibration loop on the calibration scene: Adam on (mu, xi) from (0.26, 1400) against the deposit made
    at (0.22, 1800), each iteration a smooth forward, the loss gradient and the adjoint."""
    import synth
    c = synth.make_calibration()
    dem = torch.from_numpy(c.dem).cuda()
    mask = torch.from_numpy(c.mask).cuda()
    mass = torch.from_numpy(c.mass).cuda()
    base = dict(flow_height=c.flow_height, persistence=0.9, randomness=0.16)
    P, S, seed = c.particles_per_cell, c.step_limit, c.seed
    target = avl.trajectories_smooth(dem, mask, c.cell_size, avl.Params.make(**dict(base, mu=c.mu_star, xi=c.xi_star)),
                                     P, S, seed, mass=mass).deposit
    start = avl.Params.make(**dict(base, mu=c.mu0, xi=c.xi0))
    adam = avl.Adam.make(lr_mu=0.003, lr_xi=30.0)
    avl.calibrate(dem, mask, c.cell_size, start, P, S, seed, target, 2, adam, mass=mass)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, res = avl.calibrate(dem, mask, c.cell_size, start, P, S, seed, target, iters, adam, mass=mass)
    dt = time.perf_counter() - t0
    best = int(np.argmin(hist[:, 0]))
    return {"iterations": iters, "s_total": dt, "ms_per_iteration": dt / iters * 1e3,
            "start": {"mu": c.mu0, "xi": c.xi0}, "target": {"mu": c.mu_star, "xi": c.xi_star},
            "final": {"mu": float(res.mu), "xi": float(res.xi)},
            "loss_first": float(hist[0, 0]), "loss_last": float(hist[-1, 0]),
            "best": {"iteration": best, "loss": float(hist[best, 0]), "mu": float(hist[best, 1]),
                     "xi": float(hist[best, 2])}}


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


def gradient_leg(avl, torch, reps: int) -> dict:
    """Calibration gradient: 1024^2 ridged fBm at 10 m, 5000 release cells x 128 particles, 3000 steps,
    checkpoints every 64 steps; L = MSE(deposit(mu0, xi0), deposit(mu*, xi*)). Timed: smooth forward +
    adjoint (s per gradient) against the plain forward of the same release on the same DEM."""
    import synth
    c = synth.make_calibration()
    dem = torch.from_numpy(c.dem).cuda()
    mask = torch.from_numpy(c.mask).cuda()
    mass = torch.from_numpy(c.mass).cuda()
    P, S, seed = c.particles_per_cell, c.step_limit, c.seed
    n_cells = int(c.mask.sum())
    p_star = avl.Params.make(mu=c.mu_star, xi=c.xi_star, flow_height=c.flow_height)
    p0 = avl.Params.make(mu=c.mu0, xi=c.xi0, flow_height=c.flow_height)
    target = avl.trajectories_smooth(dem, mask, c.cell_size, p_star, P, S, seed, mass=mass,
                                     max_release_cells=n_cells).deposit

    def grad_once():
        run = avl.trajectories_smooth(dem, mask, c.cell_size, p0, P, S, seed, mass=mass, max_release_cells=n_cells)
        gD = (2.0 / run.deposit.numel()) * (run.deposit - target)
        dparams, dmass, _ = avl.trajectories_backward(run, dem, mask, c.cell_size, p0, P, S, seed, gD, mass=mass)
        return run, dparams, dmass

    run, dparams, _ = grad_once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run, dparams, _ = grad_once()
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    res = None
    for _ in range(2):
        res = avl.trajectories(dem, mask, c.cell_size, p0, P, S, seed, 0, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = avl.trajectories(dem, mask, c.cell_size, p0, P, S, seed, 0, res)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    g = dparams.cpu().numpy()
    steps = int(run.stats.cpu().numpy()[0])
    return {"workload": "calibration: 1024^2 at 10 m, 5000 release cells x 128 particles, 3000 steps, "
                        "checkpoints every 64 steps, MSE of the deposit against (mu*, xi*) = (0.22, 1800)",
            "at": {"mu": c.mu0, "xi": c.xi0}, "dL_dmu": float(g[0]), "dL_dxi": float(g[1]), "dL_dh": float(g[2]),
            "particle_steps": steps, "s_per_gradient": t_grad, "ms_plain_forward": t_plain * 1e3,
            "gradient_over_plain_forward": t_grad / t_plain}


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
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
    if args.variant >= 0:
        avl.set_tuning(args.variant, True)
    if args.copy_probe:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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

    # per-step timing: the terrain passes and the trajectory call with torch events on the stream, the
    # trajectory kernel alone with the library's events around its launch on the same stream
    t_terrain = t_traj = t_kernel = 0.0
    kernel_ms = []
    avl.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        ev[2].synchronize()
        t_terrain += ev[0].elapsed_time(ev[1])
        t_traj += ev[1].elapsed_time(ev[2])
        kernel_ms.append(avl.last_kernel_ms())
        t_kernel += kernel_ms[-1]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avl.set_profiling(False)
    variant = avl.last_variant()
    # a second loop without per-step syncs gives the throughput figure
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert int(res.stats.cpu().numpy()[0]) == steps_per_pass, "particle-step count changed between passes"

    value = steps_per_pass * args.steps / elapsed
    kern_s = t_kernel / 1e3 / args.steps
    achieved_tops = OPS_PER_STEP * steps_per_pass / kern_s / 1e12
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
            "ms_trajectory_kernel": t_kernel / args.steps,
            "ms_trajectory_kernel_median": float(np.median(kernel_ms)),
            "ms_per_step_synced": wall / args.steps * 1e3,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_trajectories",
            "variant": variant,
            "achieved": achieved_tops,
            "peak": ALU_PEAK_TOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tops / ALU_PEAK_TOPS,
            "traffic": recorded_traffic(variant) if args.workload == "alpine" else None,
            "ops_per_particle_step": OPS_PER_STEP,
            "hbm_view": {"bytes_per_particle_step": BYTES_PER_STEP,
                         "achieved_GBs": BYTES_PER_STEP * steps_per_pass / kern_s / 1e9,
                         "peak_GBs": HBM_PEAK_GBS},
        },
    }
    if args.main_only:
        print(json.dumps(out), flush=True)
        return 0
    out["mipmap"] = mipmap_leg(avl, torch, res, 20)
    out["snow_cover"] = snow_leg(avl, torch, w, dem, 20)
    if args.workload == "alpine":
        out["fine_release"] = fine_leg(avl, torch, w, dem, 5)
    if not args.no_batched:
        out["batched"] = batched_leg(avl, torch, 3)
    if not args.no_gradient:
        out["gradient"] = gradient_leg(avl, torch, 5)
        out["calibration"] = calibration_leg(avl, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, mask_np, args.cpu_stride)
        if args.cpu_procs > 0:
            out["cpu_baseline"]["parallel_full_pass"] = cpu_parallel(
                w, mask_np, args.cpu_procs, res.counts.cpu().numpy(), res.vmax.cpu().numpy())
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
