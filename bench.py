#!/usr/bin/env python3
"""Benchmark of the avalanche-overlay hot path on one MI355X.

One step = one pass of the whole path over the headline workload with its DEM already resident in HBM:
normals -> release map -> release-cell list -> particle trajectories -> raster finalize. The headline is
the large region (8192^2 ridged fBm DEM at 5 m, ~1.4e6 release cells x 64 particles, step limit 8000),
the largest single-GPU workload; the tiny (256^2) and alpine (2048^2) workloads are timed as legs. The
metric is particle-steps per second (every step a particle enters counts once).

Prints one JSON line. Besides the contract fields: the roofline of the dominant kernel (the trajectory
kernel) against ceilings measured on this GPU by replaying the pass's own memory operations (its 2x2
gathers; its raster atomics without aggregation; an HBM copy), legs for the other workloads, the overlay
mipmap, snow cover, the fine release texture, batched ensembles against plain calls, gradients against
the plain forward and the calibration loop; and, on the host, the CPU oracle: a bounded single-threaded
sample, the full passes on all host threads (bit-exact check of the GPU rasters) and the FP32-vs-FP64
error of every result.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 2x2 binary32 texels read per gather (one per accepted step or stop; the release point's patch comes from
# the per-cell start records)
GATHER_BYTES = 16
# DEM gather and the two 4-byte raster updates of the model's accumulation, per particle-step
BYTES_PER_STEP = 24
HBM_PEAK_GBS = 8000.0
# Vector issue: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every 4 cycles at 2.4 GHz
# (= 39.3e12 lane-operations/s; the 157.3 TFLOP/s fp32 figure counts an FMA as 2 and packed issue as 2)
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4
# rocprofv3 figures of the trajectory kernel (recorded with the hash of the kernel sources they were taken
# on; used only while the sources are unchanged)
KERNEL_SOURCES = ["paper_2506_23364_amd/csrc/trajectories.hip", "paper_2506_23364_amd/csrc/particle.h",
                  "paper_2506_23364_amd/csrc/avl_internal.h", "paper_2506_23364_amd/build.py"]
METRIC = "particle-steps/s forward + s per (mu,xi) gradient, batched vs plain, 1 MI355X"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded(workload: str, key: str, variant: int):
    """`key[variant]` from profiles/k_trajectories_<workload>_counters.md, or None when the summary has no
    such figure or was taken on other kernel sources."""
    try:
        text = open(os.path.join(ROOT, "profiles", f"k_trajectories_{workload}_counters.md")).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and (line.startswith(key + "[") or line.startswith("source_sha256:")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    name = f"{key}[{variant}]"
    if name not in vals or vals.get("source_sha256") != kernel_source_hash():
        return None
    return float(vals[name])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["tiny", "alpine", "large"])
    ap.add_argument("--variant", type=int, default=-1,
                    help="trajectory kernel variant (default -1: the library's autotuner chooses)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads of the full-pass oracle runs (0 to skip them)")
    ap.add_argument("--main-only", action="store_true", help="only the timed passes of the headline workload")
    ap.add_argument("--leg", default="", choices=["", "roofline", "workloads", "batched", "gradient", "calibration"],
                    help="only this leg (after the headline passes); for counter runs")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched leg without the 1024 plain calls it is compared with (counter runs)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch batched calls eagerly instead of replaying captured HIP graphs (counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 256 MiB once first: a plain copy of known size that calibrates HBM byte counters")
    return ap.parse_args()


# ------------------------------------------------------------------------------------------ GPU legs

def make_inputs(torch, name):
    import synth
    w = synth.make_workload(name)
    return w, torch.from_numpy(w.dem).cuda()


def timed_passes(avl, torch, w, dem, steps: int, warmup: int) -> dict:
    """`warmup` untimed passes, then `steps` passes with per-stage events and the kernel's own events, then
    `steps` back-to-back passes for the throughput."""
    params = avl.Params.make(**w.params)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    state = {"res": None, "mask": None}

    def step(timed: bool):
        if timed:
            ev[0].record(stream)
        # normals and release map in one pass (the same bits as the two calls)
        nrm, mask = avl.normals_release_mask(dem, w.cell_size, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
        if timed:
            ev[1].record(stream)
        state["res"] = avl.trajectories(dem, mask, w.cell_size, params, w.particles_per_cell, w.step_limit, w.seed, 0,
                                        state["res"])
        if timed:
            ev[2].record(stream)
        state["mask"] = mask

    for _ in range(max(warmup, 1)):
        step(False)
    torch.cuda.synchronize()
    res = state["res"]
    stats = res.stats.cpu().numpy().astype(np.int64)
    steps_per_pass = int(stats[0])
    t_terrain = t_traj = 0.0
    kernel_ms = []
    avl.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        ev[2].synchronize()
        t_terrain += ev[0].elapsed_time(ev[1])
        t_traj += ev[1].elapsed_time(ev[2])
        kernel_ms.append(avl.last_kernel_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avl.set_profiling(False)
    variant = avl.last_variant()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    res = state["res"]
    assert int(res.stats.cpu().numpy()[0]) == steps_per_pass, "particle-step count changed between passes"
    n_release = int(state["mask"].sum().item())
    h, wd = w.dem.shape
    return {
        "res": res, "mask": state["mask"], "steps_per_pass": steps_per_pass, "variant": variant,
        "value": steps_per_pass * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
        "kernel_ms": float(np.mean(kernel_ms)),
        "config": {
            "workload": f"{w.name}: {h}x{wd} ridged diamond-square fBm DEM at {w.cell_size:g} m, release "
                        f"{w.slope_min_deg:g}-{w.slope_max_deg:g} deg above z={w.z_min:.1f} m "
                        f"({n_release} cells), {w.particles_per_cell} particles/cell, step limit {w.step_limit}, "
                        f"mu {w.params['mu']:g}, xi {w.params['xi']:g}, h {w.params['flow_height']:g}, "
                        f"persistence {w.params['persistence']:g}, randomness {w.params['randomness']:g}"
            if w.name != "tiny" else
            f"tiny: {h}x{wd} DEM at {w.cell_size:g} m, 35-degree incline with a fillet into a flat runout plus 5 m "
            f"fBm, release {w.slope_min_deg:g}-{w.slope_max_deg:g} deg above z={w.z_min:.1f} m ({n_release} cells), "
            f"{w.particles_per_cell} particles/cell, step limit {w.step_limit}, mu {w.params['mu']:g}, "
            f"xi {w.params['xi']:g}, h {w.params['flow_height']:g}",
            "release_cells": n_release,
            "particles": n_release * w.particles_per_cell,
            "particle_steps_per_pass": steps_per_pass,
            "mean_steps_per_particle": steps_per_pass / max(1, n_release * w.particles_per_cell),
            "ends_exit_stop_limit": [int(v) for v in stats[1:]],
        },
        "timing": {
            "ms_terrain_normals_mask": t_terrain / steps,
            "ms_trajectories_call": t_traj / steps,
            "ms_trajectory_kernel": float(np.mean(kernel_ms)),
            "ms_trajectory_kernel_median": float(np.median(kernel_ms)),
            "ms_per_step_synced": wall / steps * 1e3,
        },
    }


def kernel_time_ms(avl, torch, fn, reps: int) -> float:
    """Median over `reps` calls of the library's own events around the one kernel the call times."""
    ms = []
    avl.set_profiling(True)
    for _ in range(reps):
        fn()
        ms.append(avl.last_kernel_ms())
    avl.set_profiling(False)
    torch.cuda.synchronize()
    return float(np.median(ms))


def tail_probe(avl, torch, w, dem, mask, variant: int) -> dict:
    """One more pass with the library's tail probe: per block its start, the moment it finds no particle slot
    left anywhere, and its end (GPU real-time clock, 100 MHz). The tail is the time from the first block
    running out of slots to the kernel's end, during which paths started earlier finish on fewer lanes."""
    grid = avl.trajectory_grid(variant)
    buf = torch.zeros(3 * max(grid, 1), dtype=torch.uint64, device="cuda")
    avl.set_probe(buf)
    try:
        avl.trajectories(dem, mask, w.cell_size, avl.Params.make(**w.params), w.particles_per_cell, w.step_limit,
                         w.seed)
        torch.cuda.synchronize()
    finally:
        avl.set_probe(None)
    t = buf.view(torch.int64).cpu().numpy().reshape(-1, 3).astype(np.int64)
    t = t[t[:, 2] > 0]
    if t.size == 0:
        return {"blocks": 0}
    t0 = t[:, 0].min()
    ms = (t - t0) * 1e-5  # 100 MHz ticks -> ms
    dry = ms[t[:, 1] > 0, 1]
    end = ms[:, 2]
    first_dry = float(dry.min()) if dry.size else None
    return {"blocks": int(t.shape[0]), "ms_kernel_span": float(end.max()),
            "ms_first_block_out_of_slots": first_dry,
            "ms_median_block_out_of_slots": float(np.median(dry)) if dry.size else None,
            "ms_tail_after_first_out_of_slots": float(end.max() - first_dry) if dry.size else None,
            "ms_block_end_p10_p50_p90": [float(np.percentile(end, q)) for q in (10, 50, 90)],
            "tail_fraction": float((end.max() - first_dry) / end.max()) if dry.size else None}


def roofline_leg(avl, torch, w, dem, mask, run: dict, reps: int = 3) -> dict:
    """Ceilings of the trajectory kernel measured on this GPU: the pass is recorded (every particle's points
    and v^2), its 2x2 gathers and cell visits are laid out in wave order (64 neighbouring particles, step by
    step) and replayed without the model's arithmetic or dependences, and an HBM copy is timed. Each ceiling
    is the pass's work divided by the replay kernel's time."""
    params = avl.Params.make(**w.params)
    paths = avl.trajectory_paths(dem, mask, w.cell_size, params, w.particles_per_cell, w.step_limit, w.seed)
    torch.cuda.synchronize()
    same = bool(torch.equal(paths.run.counts.view(torch.int32), run["res"].counts.view(torch.int32))
                and torch.equal(paths.run.vmax, run["res"].vmax))
    ends = paths.ends.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    valid = ends != 0xFFFFFFFF
    stops = int(((ends & 3) == 2)[valid].sum().item())
    accepted = int((ends[valid] >> 2).sum().item())
    gathers = accepted + stops
    sched = avl.bench_schedule(tuple(dem.shape), paths)
    del paths
    torch.cuda.empty_cache()
    t_gather = kernel_time_ms(avl, torch, lambda: avl.bench_gather(dem, sched), reps)
    out = (torch.empty_like(run["res"].counts), torch.empty_like(run["res"].counts))
    t_atomic = kernel_time_ms(avl, torch, lambda: avl.bench_atomics(tuple(dem.shape), sched, out), reps)
    counts_equal = bool(torch.equal(out[0].view(torch.int32), run["res"].counts.view(torch.int32)))
    visits = int(sched.visits.shape[0])
    assert gathers == int(sched.gathers.numel())
    del sched, out
    torch.cuda.empty_cache()
    n_copy = 1 << 30
    src = torch.empty(n_copy, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    t_copy = kernel_time_ms(avl, torch, lambda: avl.bench_stream(src, dst), reps)
    del src, dst
    torch.cuda.empty_cache()
    steps = run["steps_per_pass"]
    t_kernel = run["kernel_ms"]
    variant = run["variant"]
    tail = tail_probe(avl, torch, w, dem, mask, variant)
    gather_ceiling = steps / (t_gather * 1e-3)
    atomic_ceiling = steps / (t_atomic * 1e-3)
    achieved = steps / (t_kernel * 1e-3)
    valu = recorded(w.name, "valu_wave_insts_per_launch", variant)
    tcc_atomic = recorded(w.name, "tcc_atomic_per_launch", variant)
    ceilings = {
        "l2_gather": {"particle_steps_per_s": gather_ceiling, "replay_ms": t_gather, "gathers": gathers,
                      "GBs": GATHER_BYTES * gathers / (t_gather * 1e-3) / 1e9},
        "atomics_unaggregated": {"particle_steps_per_s": atomic_ceiling, "replay_ms": t_atomic,
                                 "cell_visits": visits, "replay_counts_equal_pass": counts_equal,
                                 "atomics_per_s_upper": 2 * visits / (t_atomic * 1e-3)},
        "hbm_copy": {"GBs": 2 * n_copy / (t_copy * 1e-3) / 1e9, "bytes_read_and_written": 2 * n_copy,
                     "ms": t_copy, "peak_GBs": HBM_PEAK_GBS},
        "valu": None if valu is None else {
            "particle_steps_per_s": VALU_WAVE_INSTS_PER_S * steps / valu,
            "wave_insts_per_particle_step": valu / steps, "source": "rocprofv3 SQ_INSTS_VALU (profiles)"},
    }
    bound, peak_steps = "l2_gather", gather_ceiling
    achieved_bw, peak_bw = (GATHER_BYTES * gathers / (t_kernel * 1e-3) / 1e9, GATHER_BYTES * gathers / (t_gather * 1e-3) / 1e9)
    if tcc_atomic is not None:
        # the kernel's own memory-side atomics at the replay's memory-side atomic rate (the replay issues one
        # add and at most one max per visit: an upper estimate of its rate, so a ceiling on the high side);
        # each memory-side atomic moves one 32-byte request
        rate = 2.0 * visits / (t_atomic * 1e-3)
        atomic_steps = rate * steps / tcc_atomic
        ceilings["atomics_as_issued"] = {"particle_steps_per_s": atomic_steps,
                                         "memory_side_atomics_per_launch": tcc_atomic,
                                         "memory_side_atomics_per_particle_step": tcc_atomic / steps,
                                         "replay_atomics_per_s_upper": rate,
                                         "source": "rocprofv3 TCC_ATOMIC (profiles)"}
        if atomic_steps < peak_steps:
            bound, peak_steps = "atomics_as_issued", atomic_steps
            achieved_bw, peak_bw = 32 * tcc_atomic / (t_kernel * 1e-3) / 1e9, 32 * rate / 1e9
    return {
        "bound": bound, "kernel": "k_trajectories", "variant": variant, "variant_shape": avl.variant_info(variant),
        "achieved": achieved_bw, "peak": peak_bw, "unit": "GB/s",
        "frac": achieved / peak_steps,
        "traffic": recorded(w.name, "traffic_bytes_per_launch", variant),
        "achieved_particle_steps_per_s": achieved,
        "ceiling_particle_steps_per_s": peak_steps,
        "kernel_ms": t_kernel,
        "ceilings": ceilings,
        "recorded_pass_equals_timed_pass": same,
        "tail": tail,
        "hbm_view": {"bytes_per_particle_step": BYTES_PER_STEP, "achieved_GBs": BYTES_PER_STEP * steps / t_kernel / 1e6,
                     "peak_GBs": HBM_PEAK_GBS},
    }


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


def fine_leg(avl, torch, reps: int, mult: int = 2, per_texel: int = 64) -> dict:
    """The alpine tile's release rule evaluated on a release texture with mult x mult texels per DEM cell,
    with per_texel particles per release texel (mult^2 * per_texel = the plain pass's particles per cell):
    the fine release map and the trajectory pass from it."""
    w, dem = make_inputs(torch, "alpine")
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
    return {"workload": "alpine tile, release texture of 2 x 2 texels per DEM cell", "mult": mult,
            "particles_per_texel": per_texel, "release_texels": texels,
            "particles": texels * per_texel, "particle_steps_per_pass": steps,
            "ms_release_map": float(np.mean(map_ms)), "release_map_GBs": map_bytes / float(np.mean(map_ms)) / 1e6,
            "ms_trajectory_kernel": kms, "particle_steps_per_s": steps / (kms * 1e-3)}


def snow_leg(avl, torch, w, dem, reps: int) -> dict:
    """Snow-cover alpha of the DEM (section 5.1) from its normals: an HBM stream of 24 bytes per texel."""
    nrm = avl.normals(dem, w.cell_size)
    line = float(torch.quantile(dem.flatten()[::64], 0.6).item())
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


def batched_leg(avl, torch, reps: int, plain_calls: bool = True) -> dict:
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
    if not plain_calls:
        return {"runs": len(e.runs), "particle_steps": steps, "ms_batched": t_batch * 1e3,
                "particle_steps_per_s_batched": steps / t_batch, "variant": variant}
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
    plain_variant = avl.last_variant()
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
            "variant": variant, "variant_shape": avl.variant_info(variant), "plain_calls_variant": plain_variant,
            "batched_equals_plain": same}


def gradient_case(avl, torch, dem_np, mask_np, mass_np, cs, target_params, p0, P, S, seed, reps):
    """s per (mu, xi) gradient (smooth forward + MSE gradient + adjoint) against the plain forward of the same
    release; returns the timings, the GPU gradient and the raster gradient gD for the host checks."""
    dem = torch.from_numpy(dem_np).cuda()
    mask = torch.from_numpy(mask_np).cuda()
    mass = torch.from_numpy(mass_np).cuda()
    n_cells = int(mask_np.sum())
    target = avl.trajectories_smooth(dem, mask, cs, avl.Params.make(**target_params), P, S, seed, mass=mass,
                                     max_release_cells=n_cells).deposit
    pp = avl.Params.make(**p0)

    def grad_once():
        run = avl.trajectories_smooth(dem, mask, cs, pp, P, S, seed, mass=mass, max_release_cells=n_cells)
        gD = (2.0 / run.deposit.numel()) * (run.deposit - target)
        dparams, dmass, _ = avl.trajectories_backward(run, dem, mask, cs, pp, P, S, seed, gD, mass=mass)
        return run, dparams, gD

    run, dparams, gD = grad_once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run, dparams, gD = grad_once()
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    res = None
    for _ in range(2):
        res = avl.trajectories(dem, mask, cs, pp, P, S, seed, 0, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = avl.trajectories(dem, mask, cs, pp, P, S, seed, 0, res)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    g = dparams.cpu().numpy()
    steps = int(run.stats.cpu().numpy()[0])
    n_part = n_cells * P
    return ({"dL_dmu": float(g[0]), "dL_dxi": float(g[1]), "dL_dh": float(g[2]), "particle_steps": steps,
             "mean_steps_per_particle": steps / max(1, n_part), "checkpoint_segments_max": -(-S // 64),
             "s_per_gradient": t_grad, "ms_plain_forward": t_plain * 1e3, "gradient_over_plain_forward": t_grad / t_plain},
            g, gD.float().cpu().numpy())


def gradient_leg(avl, torch, reps: int) -> tuple[dict, dict]:
    """Calibration gradient (1024^2 at 10 m, 5000 release cells x 128 particles, 3000 steps, checkpoints every 64
    steps; L = MSE(deposit(mu0, xi0), deposit(mu*, xi*))), and the same on the tiny workload's release, whose paths
    run ~130 steps (several checkpoint segments): s per gradient against the plain forward."""
    import oracle
    import synth
    c = synth.make_calibration()
    base = dict(flow_height=c.flow_height)
    out, g, gD = gradient_case(avl, torch, c.dem, c.mask, c.mass, c.cell_size, dict(base, mu=c.mu_star, xi=c.xi_star),
                               dict(base, mu=c.mu0, xi=c.xi0), c.particles_per_cell, c.step_limit, c.seed, reps)
    out["workload"] = ("calibration: 1024^2 at 10 m, 5000 release cells x 128 particles, 3000 steps, checkpoints every "
                       "64 steps, MSE of the deposit against (mu*, xi*) = (0.22, 1800)")
    out["at"] = {"mu": c.mu0, "xi": c.xi0}
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, w.cell_size), w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min,
                               w.z_max)
    tp = dict(w.params)
    long_out, g_long, gD_long = gradient_case(
        avl, torch, w.dem, mask, mask.astype(np.float32), w.cell_size, dict(tp, mu=0.22, xi=1800.0),
        dict(tp, mu=w.params["mu"], xi=w.params["xi"]), w.particles_per_cell, w.step_limit, w.seed, reps)
    long_out["workload"] = (f"long paths: the tiny workload's release ({int(mask.sum())} cells x {w.particles_per_cell} "
                            f"particles, step limit {w.step_limit}), mass 1 per cell, MSE against the deposit at "
                            f"(0.22, 1800), gradient at (mu, xi) = ({w.params['mu']:g}, {w.params['xi']:g})")
    out["long_paths"] = long_out
    host = {"calibration": (c, g, gD), "long": (w, mask, g_long, gD_long)}
    return out, host


# ------------------------------------------------------------------------------------------ host (oracle) legs

def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def oracle_sample(w, mask: np.ndarray, steps_per_pass: int, seconds: float = 10.0) -> dict:
    """The FP32 oracle, single-threaded, on every `stride`-th release cell (stride chosen for ~`seconds` of work
    at ~26 M particle-steps/s)."""
    import oracle
    stride = max(1, int(round(steps_per_pass / (26e6 * seconds))))
    cells = np.flatnonzero(mask)
    sample = np.zeros(mask.size, np.uint8)
    sample[cells[::stride]] = 1
    sample = sample.reshape(mask.shape)
    p = oracle.make_params(**w.params)
    t0 = time.perf_counter()
    res = oracle.trajectories(w.dem, sample, w.cell_size, p, w.particles_per_cell, w.step_limit, w.seed)
    dt = time.perf_counter() - t0
    return {"value": res.steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.name}: 1 in {stride} release cells ({int(sample.sum())} cells x {w.particles_per_cell} "
                      f"particles, {res.steps} particle-steps, {dt:.1f} s, single-threaded FP32 C oracle)"}


def oracle_full_pass(w, mask: np.ndarray, prec: str, threads: int):
    """The whole pass on the oracle in `threads` host threads (the C calls release the GIL), each taking chunks
    of consecutive release cells into rasters of its own; the rasters are merged exactly at the end (counts
    add, speeds take the maximum)."""
    import queue
    import threading
    import oracle
    oracle._lib(prec)  # load the library once, before the threads
    cells = np.flatnonzero(mask)
    todo = queue.Queue()
    for c in np.array_split(cells, max(1, 4 * threads)):
        if c.size:
            todo.put(c)
    p = oracle.make_params(**w.params)
    real = np.float32 if prec == "f32" else np.float64
    acc = []

    def worker():
        counts = np.zeros(mask.shape, np.uint64)
        vmax = np.zeros(mask.shape, real)
        steps = 0
        m = np.zeros(mask.size, np.uint8)
        while True:
            try:
                chunk = todo.get_nowait()
            except queue.Empty:
                break
            m[:] = 0
            m[chunk] = 1
            r = oracle.trajectories(w.dem, m.reshape(mask.shape), w.cell_size, p, w.particles_per_cell,
                                    w.step_limit, w.seed, prec=prec)
            counts += r.counts
            np.maximum(vmax, r.vmax, out=vmax)
            steps += r.steps
        acc.append((counts, vmax, steps))

    t0 = time.perf_counter()
    ts = [threading.Thread(target=worker) for _ in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    counts = np.zeros(mask.shape, np.uint64)
    vmax = np.zeros(mask.shape, real)
    steps = 0
    for c, v, s in acc:
        counts += c
        np.maximum(vmax, v, out=vmax)
        steps += s
    return counts, vmax, steps, dt


def fp64_error(c32, v32, s32, c64, v64, s64) -> dict:
    """FP32 against FP64 oracle results of the same pass (paths diverge where a rounding moves a step across a
    texel edge, so the rasters differ by more than the rounding of v)."""
    vis32, vis64 = c32 > 0, c64 > 0
    v32d = v32.astype(np.float64)
    pos = vis32 & vis64 & (v32d > 0) & (v64 > 0)
    rel = np.abs(v32d - v64)[pos] / v64[pos]
    return {"count_cells_differing": int((c32 != c64).sum()), "cells_visited_fp32": int(vis32.sum()),
            "visited_set_symmetric_difference": int((vis32 ^ vis64).sum()),
            "entries_fp32": int(c32.sum()), "entries_fp64": int(c64.sum()),
            "max_abs_count_difference": int(np.abs(c32.astype(np.int64) - c64.astype(np.int64)).max()),
            "vmax_max_rel_difference": float(rel.max()) if rel.size else 0.0,
            "vmax_median_rel_difference": float(np.median(rel)) if rel.size else 0.0,
            "vmax_cells_rel_difference_above_1e-5": int((rel > 1e-5).sum()),
            "vmax_cells_zero_in_one_precision_only": int(((vis32 & vis64) & ((v32d > 0) != (v64 > 0))).sum()),
            "particle_steps_fp32": int(s32), "particle_steps_fp64": int(s64)}


def oracle_workload_checks(w, mask, gpu_counts, gpu_vmax, threads: int) -> dict:
    c32, v32, s32, t32 = oracle_full_pass(w, mask, "f32", threads)
    c64, v64, s64, t64 = oracle_full_pass(w, mask, "f64", threads)
    return {"full_pass_fp32": {"value": s32 / t32, "unit": "particle-steps/s", "threads": threads, "seconds": t32,
                               "particle_steps": int(s32),
                               "gpu_rasters_equal_oracle": bool(np.array_equal(c32.astype(np.uint32), gpu_counts)
                                                                and np.array_equal(v32, gpu_vmax))},
            "fp64_seconds": t64,
            "fp32_vs_fp64": fp64_error(c32, v32, s32, c64, v64, s64)}


def gradient_fp64_checks(host: dict) -> dict:
    """GPU gradients against the FP64 oracle's on the same raster gradient gD; the share of particles whose
    binary32 path differs from binary64; and the whole loss's central difference (steps of 1e-3 of the parameter,
    jumps of particles whose end changes included) against the pathwise FP64 gradient."""
    import oracle
    out = {}
    c, g, gD = host["calibration"]
    w, mask, g_long, gD_long = host["long"]
    cases = {
        "calibration": (c.dem, c.mask, c.mass, c.cell_size, dict(mu=c.mu0, xi=c.xi0, flow_height=c.flow_height),
                        c.particles_per_cell, c.step_limit, c.seed, g, gD, True),
        "long_paths": (w.dem, mask, mask.astype(np.float32), w.cell_size, dict(w.params), w.particles_per_cell,
                       w.step_limit, w.seed, g_long, gD_long, False),
    }
    for name, (dem, m, mass, cs, p0, P, S, seed, g_gpu, gD_np, jump) in cases.items():
        op = oracle.make_params(**p0)
        g64 = oracle.smooth_backward(dem, m, cs, op, P, S, seed, gD_np, mass=mass, prec="f64")
        _, r32, s32 = oracle.smooth_particles(dem, m, cs, op, P, S, seed, gD_np, mass=mass, prec="f32")
        _, r64, s64 = oracle.smooth_particles(dem, m, cs, op, P, S, seed, gD_np, mass=mass, prec="f64")
        same = (r32 == r64) & (s32 == s64)
        ref = (g64.dmu, g64.dxi, g64.dh)
        d = {"fp32_paths_differing_fraction": float(1.0 - same.mean()),
             "dL_dmu_fp64": ref[0], "dL_dxi_fp64": ref[1], "dL_dh_fp64": ref[2]}
        for i, nm in enumerate(("mu", "xi", "h")):
            d[f"rel_err_dL_d{nm}"] = abs(float(g_gpu[i]) - ref[i]) / abs(ref[i]) if ref[i] else None
        if jump:
            gl = gD_np.astype(np.float64)
            for nm in ("mu", "xi"):
                h = 1e-3 * p0[nm]
                L = [float((gl * oracle.smooth_forward(dem, m, cs, oracle.make_params(**dict(p0, **{nm: p0[nm] + s * h})),
                                                       P, S, seed, mass=mass, prec="f64").dep).sum()) for s in (1, -1)]
                fd = (L[0] - L[1]) / (2 * h)
                k = ("mu", "xi").index(nm)
                d[f"whole_loss_central_difference_dL_d{nm}"] = fd
                d[f"jump_part_dL_d{nm}"] = (fd - ref[k]) / fd
        out[name] = d
    return out


# ------------------------------------------------------------------------------------------ main

def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "detail": "particles are independent; a multi-GPU run would split particle ranges and "
                                    "all-reduce the integer rasters (see the design notes)"}))
        return 2
    import torch
    import paper_2506_23364_amd as avl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    torch.cuda.set_device(0)
    if args.variant >= 0 or args.no_graphs:
        avl.set_tuning(args.variant, not args.no_graphs)
    if args.copy_probe:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w, dem = make_inputs(torch, args.workload)
    run = timed_passes(avl, torch, w, dem, args.steps, args.warmup)
    steps_per_pass = run["steps_per_pass"]
    kern_s = run["kernel_ms"] * 1e-3
    out = {
        "metric": METRIC,
        "value": run["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": run["config"],
        "timing": run["timing"],
        "roofline": {"bound": None, "note": "ceilings are measured by the roofline leg (not run with --main-only)",
                     "kernel": "k_trajectories", "variant": run["variant"],
                     "achieved_particle_steps_per_s": steps_per_pass / kern_s,
                     "hbm_view": {"bytes_per_particle_step": BYTES_PER_STEP,
                                  "achieved_GBs": BYTES_PER_STEP * steps_per_pass / kern_s / 1e9,
                                  "peak_GBs": HBM_PEAK_GBS}},
    }
    if args.main_only:
        print(json.dumps(out), flush=True)
        return 0
    only = args.leg
    if only in ("", "roofline"):
        out["roofline"] = roofline_leg(avl, torch, w, dem, run["mask"], run)
    if only == "":
        out["mipmap"] = mipmap_leg(avl, torch, run["res"], 20)
        out["snow_cover"] = snow_leg(avl, torch, w, dem, 20)
    host_runs = {args.workload: (w, run)}
    if only in ("", "workloads"):
        out["workloads"] = {}
        for name in ("tiny", "alpine", "large"):
            if name == args.workload:
                continue
            w2, dem2 = make_inputs(torch, name)
            r2 = timed_passes(avl, torch, w2, dem2, args.steps, args.warmup)
            leg = {k: r2[k] for k in ("value", "ms_per_step", "config", "timing", "variant")}
            leg["unit"] = "particle-steps/s"
            leg["roofline"] = roofline_leg(avl, torch, w2, dem2, r2["mask"], r2)
            out["workloads"][name] = leg
            host_runs[name] = (w2, r2)
            del dem2
    if only == "":
        out["fine_release"] = fine_leg(avl, torch, 5)
    if only in ("", "batched"):
        out["batched"] = batched_leg(avl, torch, 3, not args.no_plain)
    grad_host = None
    if only in ("", "gradient"):
        out["gradient"], grad_host = gradient_leg(avl, torch, 5)
    if only in ("", "calibration"):
        out["calibration"] = calibration_leg(avl, torch)
    if not args.no_cpu_baseline and only == "":
        mask_np = run["mask"].cpu().numpy()
        base = oracle_sample(w, mask_np, steps_per_pass)
        base.update({"cpu": cpu_model(), "os_cpu_count": os.cpu_count(), "threads_full_pass": args.cpu_threads})
        if args.cpu_threads > 0:
            base["workloads"] = {}
            for name, (w2, r2) in host_runs.items():
                base["workloads"][name] = oracle_workload_checks(
                    w2, r2["mask"].cpu().numpy(), r2["res"].counts.cpu().numpy(), r2["res"].vmax.cpu().numpy(),
                    args.cpu_threads)
        if grad_host is not None:
            base["gradient_fp32_vs_fp64"] = gradient_fp64_checks(grad_host)
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
