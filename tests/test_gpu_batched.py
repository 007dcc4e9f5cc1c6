"""GPU parity of the batched ensemble entry point (avl_trajectories_batched) and of the kernel variants.

Every run of a batch is defined as the plain trajectory pass of its (tile, scenario, parameter set,
seed, run id), so each run's rasters and statistics must equal the oracle's plain run bit for bit
(max velocity within 1e-5 relative). Every autotuner variant must give identical results, and graph
replays (with new parameter values written to device memory between replays) must match eager runs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

INF = float("inf")


@pytest.fixture(scope="module")
def avl():
    import paper_2506_23364_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield m
    m.set_tuning(-1, True)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small_ensemble():
    rng = np.random.default_rng(44)
    dems = np.stack([synth.alpine_dem(128, 900.0, seed=60 + t)[:97, :83] for t in range(3)]).astype(np.float32)
    masks = []
    for t in range(3):
        sl = synth.slope_deg(dems[t], 10.0)
        m = ((sl >= 25) & (sl <= 50) & (dems[t] >= np.quantile(dems[t], 0.5))).astype(np.uint8)
        keep = rng.random(m.shape) < [0.5, 0.2, 0.05][t]
        masks.append((m & keep).astype(np.uint8))
    masks.append(np.zeros_like(masks[0]))  # an empty scenario
    masks = np.stack(masks)
    params = [dict(synth.DEFAULT_PARAMS, mu=0.2, xi=2000.0),
              dict(synth.DEFAULT_PARAMS, mu=0.12, xi=INF, randomness=0.3),
              dict(synth.DEFAULT_PARAMS, mu=0.35, xi=600.0, flow_height=2.5, step_cells=0.7),
              dict(synth.DEFAULT_PARAMS, mu=0.05, tan_alpha=0.45, persistence=0.6)]
    runs = []
    for t in range(3):
        for s in range(4):
            for p in range(4):
                if (t + s + p) % 3 == 0:
                    runs.append((t, s, p, 1000 + len(runs), 0x1234567890ABCDEF + t))
    return dems, masks, params, runs


def oracle_run(dems, masks, params, run, P, S):
    t, s, p, run_id, seed = run
    return oracle.trajectories(dems[t], masks[s], 10.0, oracle.make_params(**params[p]), P, S, seed, run_id)


def check_batch(res, dems, masks, params, runs, P, S, label=""):
    counts, vmax, stats, status = host(res.counts), host(res.vmax), host(res.stats), host(res.status)
    for k, run in enumerate(runs):
        ref = oracle_run(dems, masks, params, run, P, S)
        assert status[k] == 0
        assert np.array_equal(counts[k], ref.counts), f"{label} run {k}"
        np.testing.assert_allclose(vmax[k], ref.vmax, rtol=1e-5, atol=0, err_msg=f"{label} run {k}")
        assert list(stats[k]) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit], f"{label} run {k}"


def run_batch(avl, dems, masks, params, runs, P, S, out=None):
    d = torch.from_numpy(dems).cuda()
    m = torch.from_numpy(masks).cuda()
    return avl.trajectories_batched(d, m, 10.0, avl.params_tensor(params, "cuda"), avl.runs_tensor(runs, "cuda"), P, S,
                                    out)


def test_batch_equals_plain_oracle_runs(avl):
    dems, masks, params, runs = small_ensemble()
    res = run_batch(avl, dems, masks, params, runs, 5, 300)
    check_batch(res, dems, masks, params, runs, 5, 300, "eager default stream")


def test_batch_bad_runs_are_flagged(avl):
    dems, masks, params, runs = small_ensemble()
    bad_params = params + [dict(synth.DEFAULT_PARAMS, mu=-1.0)]
    runs2 = [runs[0], (7, 0, 0, 1, 1), (0, 9, 0, 1, 1), (0, 0, 11, 1, 1), (0, 0, 4, 1, 1), runs[1]]
    res = run_batch(avl, dems, masks, bad_params, runs2, 3, 100)
    status = host(res.status)
    assert list(status) == [0, 1, 1, 1, 2, 0]
    counts = host(res.counts)
    assert counts[1:5].sum() == 0
    for k in (0, 5):
        ref = oracle_run(dems, masks, bad_params, runs2[k], 3, 100)
        assert np.array_equal(counts[k], ref.counts)


def test_start_records_owner_and_other_tiles(avl):
    """Start states of a scenario are recorded on the tile of its first valid run and read by the runs on
    that tile; runs that pair the scenario with another tile compute them. Here scenario 0's first run is
    invalid (bad parameters), so its records belong to the second run's tile (2); runs on tiles 0 and 1
    compute, and every valid run equals the oracle."""
    dems, masks, params, runs = small_ensemble()
    ps = params + [dict(synth.DEFAULT_PARAMS, mu=-1.0)]
    runs2 = [(0, 0, 4, 50, 9), (2, 0, 0, 51, 9), (0, 0, 1, 52, 9), (2, 0, 2, 53, 9), (1, 0, 3, 54, 9),
             (2, 1, 0, 55, 9)]
    res = run_batch(avl, dems, masks, ps, runs2, 4, 300)
    status = host(res.status)
    assert list(status) == [2, 0, 0, 0, 0, 0]
    valid = [(k, r) for k, r in enumerate(runs2) if status[k] == 0]
    counts, vmax, stats = host(res.counts), host(res.vmax), host(res.stats)
    for k, run in valid:
        ref = oracle_run(dems, masks, ps, run, 4, 300)
        assert np.array_equal(counts[k], ref.counts), f"run {k}"
        np.testing.assert_allclose(vmax[k], ref.vmax, rtol=1e-5, atol=0, err_msg=f"run {k}")
        assert list(stats[k]) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit], f"run {k}"
    assert counts[0].sum() == 0


def test_every_variant_gives_identical_rasters(avl):
    dems, masks, params, runs = small_ensemble()
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, 10.0), w.dem, 30, 45, w.z_min, w.z_max)
    dem_t, mask_t = torch.from_numpy(w.dem).cuda(), torch.from_numpy(mask).cuda()
    ref_b = ref_p = None
    try:
        for v in range(avl.tuning_variants()):
            avl.set_tuning(v, True)
            res = run_batch(avl, dems, masks, params, runs, 4, 200)
            got_b = [host(res.counts), host(res.vmax), host(res.stats)]
            assert avl.last_variant() == v
            r = avl.trajectories(dem_t, mask_t, 10.0, avl.Params.make(**w.params), 4, 500, 3)
            got_p = [host(r.counts), host(r.vmax), host(r.stats)]
            if ref_b is None:
                ref_b, ref_p = got_b, got_p
            for a, b in zip(got_b + got_p, ref_b + ref_p):
                assert np.array_equal(a, b), f"variant {v}"
    finally:
        avl.set_tuning(-1, True)
    ref = oracle.trajectories(w.dem, mask, 10.0, oracle.make_params(**w.params), 4, 500, 3)
    assert np.array_equal(ref_p[0], ref.counts)


def cone_scene():
    """16 x 16 cone (8 m of height per cell of radius, ~39 degrees) with a pit of four cells at its
    centre; the 32 cells within 3 cells of the axis release."""
    yy, xx = np.mgrid[0:16, 0:16].astype(np.float64)
    r = np.sqrt((xx - 7.5) ** 2 + (yy - 7.5) ** 2)
    return (r * 8.0).astype(np.float32), (r < 3.0).astype(np.uint8)


def test_table_retention_every_variant(avl):
    """The accumulation table may keep a busy cell's slot from one epoch to the next, its count held in 16
    bits until it reaches the rasters. On a cone every path ends in the pit: at 2,000 particles per cell
    every variant equals the oracle; at 1,000,000 per cell (32 M particles, a full grid) the blocks enter a
    pit cell more often than a retained count may reach, and every variant must equal the one without
    retention."""
    dem, mask = cone_scene()
    d, m = torch.from_numpy(dem).cuda(), torch.from_numpy(mask).cuda()
    p = dict(synth.DEFAULT_PARAMS)
    ref = oracle.trajectories(dem, mask, 10.0, oracle.make_params(**p), 2000, 200, 5)
    try:
        for v in range(avl.tuning_variants()):
            avl.set_tuning(v, True)
            r = avl.trajectories(d, m, 10.0, avl.Params.make(**p), 2000, 200, 5)
            assert np.array_equal(host(r.counts), ref.counts), f"variant {v}"
            np.testing.assert_allclose(host(r.vmax), ref.vmax, rtol=1e-5, atol=0, err_msg=f"variant {v}")
            assert list(host(r.stats)) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit], f"variant {v}"
        outs = []
        for v in range(avl.tuning_variants()):
            avl.set_tuning(v, True)
            r = avl.trajectories(d, m, 10.0, avl.Params.make(**p), 1_000_000, 200, 5)
            outs.append([host(r.counts), host(r.vmax), host(r.stats)])
        counts = outs[0][0]
        # 512 blocks: some block enters the pit cell more often than a retained count may reach (2^15)
        assert int(counts.max()) > 512 * 32768, int(counts.max())
        assert int(outs[0][2][0]) > 32_000_000
        plain = outs[4]  # variant 4 keeps no slot across epochs and counts in 32 bits
        for v, o in enumerate(outs):
            for a, b in zip(o, plain):
                assert np.array_equal(a, b), f"variant {v}"
    finally:
        avl.set_tuning(-1, True)


def test_graph_replay_with_new_parameters(avl):
    dems, masks, params, runs = small_ensemble()
    d = torch.from_numpy(dems).cuda()
    m = torch.from_numpy(masks).cuda()
    ptab = avl.params_tensor(params, "cuda")
    rtab = avl.runs_tensor(runs, "cuda")
    stream = torch.cuda.Stream()
    out = None
    variants = [params,
                [dict(p, mu=p["mu"] + 0.03) for p in params],
                [dict(p, randomness=0.05) for p in params]]
    with torch.cuda.stream(stream):
        for rep in range(2):
            for vi, pv in enumerate(variants):
                ptab.copy_(avl.params_tensor(pv, "cuda"))
                out = avl.trajectories_batched(d, m, 10.0, ptab, rtab, 4, 250, out)
                stream.synchronize()
                # unrelated eager work between replays
                junk = torch.randn(1 << 20, device="cuda").sum()
                check_batch(out, dems, masks, pv, runs, 4, 250, f"replay {rep} params {vi}")
                del junk
    # the same with graphs off
    avl.set_tuning(-1, False)
    try:
        with torch.cuda.stream(stream):
            res = avl.trajectories_batched(d, m, 10.0, avl.params_tensor(variants[1], "cuda"), rtab, 4, 250)
            stream.synchronize()
        check_batch(res, dems, masks, variants[1], runs, 4, 250, "graphs off")
    finally:
        avl.set_tuning(-1, True)


def test_ensemble_full_size(avl):
    """The full 16-tile x 64-parameter ensemble (1024 runs, 1024^2 tiles, 32 particles per cell, 2000 steps) in
    the launch shape the benchmark times: every run against the oracle's plain run of its (tile, scenario,
    parameter set, seed, run id), run on all host threads, counts and statistics bit for bit and speeds within
    1e-5 (so the largest scenarios, up to 26,397 release cells, are checked as well as the smallest)."""
    from support import oracle_threads
    e = synth.make_ensemble()
    d = torch.from_numpy(e.dems).cuda()
    m = torch.from_numpy(e.masks).cuda()
    res = avl.trajectories_batched(d, m, e.cell_size, avl.params_tensor(e.params, "cuda"),
                                   avl.runs_tensor(e.runs, "cuda"), e.particles_per_cell, e.step_limit)
    stats = host(res.stats)
    assert (host(res.status) == 0).all()
    counts = host(res.counts)
    vmax = host(res.vmax)
    sizes = e.masks.sum(axis=(1, 2))
    print(f"ensemble: {len(e.runs)} runs, scenarios {sizes.min()}-{sizes.max()} cells, oracle on "
          f"{oracle_threads.host_threads()} threads", flush=True)

    def check(k):
        t, sc, p, run_id, seed = e.runs[k]
        ref = oracle.trajectories(e.dems[t], e.masks[sc], e.cell_size, oracle.make_params(**e.params[p]),
                                  e.particles_per_cell, e.step_limit, seed, run_id)
        ok_c = np.array_equal(counts[k], ref.counts)
        ok_v = np.allclose(vmax[k], ref.vmax, rtol=1e-5, atol=0)
        ok_s = list(stats[k]) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit]
        return ok_c and ok_v and ok_s

    ok = oracle_threads.run_all(range(len(e.runs)), check)
    bad = [k for k, v in enumerate(ok) if not v]
    assert not bad, f"runs differing from the oracle: {bad[:20]}"
    ends = stats[:, 1:].sum(axis=1)
    expect = np.array([sizes[r[1]] * e.particles_per_cell for r in e.runs])
    assert np.array_equal(ends, expect)
