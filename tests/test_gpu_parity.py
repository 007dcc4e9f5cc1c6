"""GPU parity: the HIP path (called through the C ABI) against the CPU oracle on the same seeded inputs.

Bar (bit-exact for integer work, stated tolerance for floats):
  * normals nx, ny, nz: bit-exact (same binary32 operations); slope channel within 4e-5 degrees;
  * release mask and release-cell list: bit-exact;
  * hit counts, visited set, step / end statistics: bit-exact;
  * max velocity: within 1e-5 relative per cell (the arithmetic is the same, so it is expected exact).
Sizes span several tiles and a ragged tail; the full-size alpine tile is checked on a deterministic
sample of release cells (the oracle runs the sample, the GPU the sample and its complement, and the
full run must equal their sum).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

INF = float("inf")
VMAX_RTOL = 1e-5


@pytest.fixture(scope="module")
def avl():
    import paper_2506_23364_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_run(avl, dem, mask, cs, params: dict, P, S, seed, run=0):
    res = avl.trajectories(dev(dem), dev(mask), cs, avl.Params.make(**params), P, S, seed, run)
    return host(res.counts), host(res.vmax), host(res.stats)


def assert_run_equal(got, ref, label=""):
    counts, vmax, stats = got
    assert np.array_equal(counts, ref.counts), f"{label}: counts differ at {np.argwhere(counts != ref.counts)[:5]}"
    assert np.array_equal(counts > 0, ref.counts > 0)
    np.testing.assert_allclose(vmax, ref.vmax, rtol=VMAX_RTOL, atol=0, err_msg=label)
    assert list(stats) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit], label


def both(avl, dem, mask, cs, params, P, S, seed, run=0, label=""):
    ref = oracle.trajectories(dem, mask, cs, oracle.make_params(**params), P, S, seed, run)
    got = gpu_run(avl, dem, mask, cs, params, P, S, seed, run)
    assert_run_equal(got, ref, label)
    return got, ref


# ------------------------------------------------------------------------------------------ terrain

def _terrain_cases():
    rng = np.random.default_rng(5)
    return [
        ("tiny", synth.incline_fillet_dem(256, 10.0, seed=1), 10.0),
        ("ragged_37x53", (rng.standard_normal((37, 53)) * 30).astype(np.float32), 7.5),
        ("2x2", np.array([[0, 1], [3, 7]], np.float32), 2.0),
        ("1000x3", (rng.standard_normal((1000, 3)) * 5).astype(np.float32), 1.0),
        ("alpine_2048", synth.make_workload("alpine").dem, 10.0),
    ]


@pytest.mark.parametrize("case", range(5), ids=[c[0] for c in _terrain_cases()])
def test_normals_mask_cells_bitexact(avl, case):
    name, dem, cs = _terrain_cases()[case]
    ref_n = oracle.normals(dem, cs)
    got_n = host(avl.normals(dev(dem), cs))
    assert np.array_equal(got_n[..., :3], ref_n[..., :3]), name
    assert np.max(np.abs(got_n[..., 3] - ref_n[..., 3])) < 4e-5
    zlo = float(np.quantile(dem, 0.3))
    for smin, smax, zmin, zmax in ((30.0, 45.0, zlo, INF), (0.0, 90.0, -INF, INF), (10.0, 20.0, -INF, zlo)):
        ref_m = oracle.release_mask(ref_n, dem, smin, smax, zmin, zmax)
        got_m = host(avl.release_mask(dev(got_n), dev(dem), smin, smax, zmin, zmax))
        assert np.array_equal(got_m, ref_m), (name, smin, smax)
        # the one-pass call writes exactly what the two calls write
        fn, fm = avl.normals_release_mask(dev(dem), cs, smin, smax, zmin, zmax)
        assert np.array_equal(host(fn).view(np.uint32), got_n.view(np.uint32)), (name, "fused normals")
        assert np.array_equal(host(fm), ref_m), (name, smin, smax, "fused mask")
        cells, n = avl.release_cells(dev(ref_m))
        n = int(host(n)[0])
        ref_c = oracle.compact(ref_m)
        assert n == len(ref_c)
        assert np.array_equal(host(cells)[:n], ref_c)


@pytest.mark.parametrize("offset", [1, 3, 8])
def test_release_cells_unaligned_mask(avl, offset):
    # a mask that starts off a 16-byte boundary takes the byte-wise reads
    rng = np.random.default_rng(offset)
    m = (rng.random((97, 131)) < 0.3).astype(np.uint8)
    buf = torch.zeros(m.size + offset, dtype=torch.uint8, device="cuda")
    view = buf[offset:].view(m.shape)
    view.copy_(torch.from_numpy(m))
    assert view.data_ptr() % 16 != 0
    cells, n = avl.release_cells(view)
    n = int(host(n)[0])
    ref = oracle.compact(m)
    assert n == len(ref)
    assert np.array_equal(host(cells)[:n], ref)


@pytest.mark.parametrize("p", [0.0, 0.001, 0.5, 1.0])
def test_release_cells_density(avl, p):
    rng = np.random.default_rng(int(p * 1000) + 1)
    m = (rng.random((333, 517)) < p).astype(np.uint8)
    cells, n = avl.release_cells(dev(m))
    n = int(host(n)[0])
    assert n == int(m.sum())
    assert np.array_equal(host(cells)[:n], np.flatnonzero(m))


# ------------------------------------------------------------------------------------------ trajectories

def test_tiny_workload_full(avl):
    w = synth.make_workload("tiny")
    nrm = oracle.normals(w.dem, w.cell_size)
    mask = oracle.release_mask(nrm, w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    (counts, vmax, stats), ref = both(avl, w.dem, mask, w.cell_size, w.params, w.particles_per_cell, w.step_limit,
                                      w.seed, 0, "tiny")
    assert ref.steps > 3e7
    # the whole pipeline from the DEM gives the same result
    _, m2, res = avl.overlay(dev(w.dem), w.cell_size, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max,
                             avl.Params.make(**w.params), w.particles_per_cell, w.step_limit, w.seed)
    assert np.array_equal(host(m2), mask)
    assert np.array_equal(host(res.counts), ref.counts)
    # and it is reproducible bit for bit
    again = gpu_run(avl, w.dem, mask, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    assert np.array_equal(again[0], counts) and np.array_equal(again[1], vmax) and np.array_equal(again[2], stats)


def _param_grid():
    base = dict(mu=0.2, xi=2000.0, flow_height=1.0, persistence=0.9, randomness=0.16, step_cells=1.0, tan_alpha=-1.0)
    yield "default", base
    yield "no_drag", dict(base, xi=INF)
    yield "no_random", dict(base, randomness=0.0)
    yield "straight", dict(base, persistence=1.0, randomness=0.0)
    yield "steepest", dict(base, persistence=0.0, randomness=0.0)
    yield "half_step", dict(base, step_cells=0.5, randomness=0.4)
    yield "long_step", dict(base, step_cells=2.5)
    yield "runout_angle", dict(base, mu=0.05, tan_alpha=math.tan(math.radians(25.0)))
    yield "frictionless", dict(base, mu=0.0, xi=INF)
    yield "thick_flow", dict(base, mu=0.35, xi=600.0, flow_height=3.0, randomness=0.5)


@pytest.mark.parametrize("name,params", list(_param_grid()), ids=[n for n, _ in _param_grid()])
def test_ragged_grid_param_grid(avl, name, params):
    dem = synth.alpine_dem(128, 900.0, seed=31)[:101, :77].copy()
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 25.0, 50.0, float(np.quantile(dem, 0.5)), INF)
    assert mask.sum() > 50
    both(avl, dem, mask, 10.0, params, 7, 600, 0xDEADBEEF12345678, 3, name)


def test_reused_rasters_after_a_faster_pass(avl):
    """The max check before a raster max reads the cell as the caches hold it. Rasters that a previous pass
    left with larger speeds (low friction) are reused by a pass with smaller ones, on every trajectory
    variant: a value cached from the earlier pass would skip maxima and leave cells too low, so each second
    pass must still equal the oracle."""
    dem = synth.alpine_dem(160, 900.0, seed=41)
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 28.0, 45.0, float(np.quantile(dem, 0.4)), INF)
    fast = dict(synth.DEFAULT_PARAMS, mu=0.02, xi=8000.0)
    slow = dict(synth.DEFAULT_PARAMS, mu=0.3, xi=800.0)
    ref_slow = oracle.trajectories(dem, mask, 10.0, oracle.make_params(**slow), 8, 800, 21)
    d, m = dev(dem), dev(mask)
    try:
        for v in range(avl.tuning_variants()):
            avl.set_tuning(v, True)
            res = avl.trajectories(d, m, 10.0, avl.Params.make(**fast), 8, 800, 21)
            fast_vmax = host(res.vmax)
            res = avl.trajectories(d, m, 10.0, avl.Params.make(**slow), 8, 800, 21, 0, res)
            got = (host(res.counts), host(res.vmax), host(res.stats))
            assert fast_vmax.max() > got[1].max()
            assert_run_equal(got, ref_slow, f"variant {v}")
    finally:
        avl.set_tuning(-1, True)


def test_bruteforce_8x8_cases(avl):
    rng = np.random.default_rng(8)
    for case in range(24):
        r = np.arange(8, dtype=np.float64)[:, None]
        dem = (np.broadcast_to(rng.uniform(2, 9) * (8 - r), (8, 8)) + rng.standard_normal((8, 8)) * rng.uniform(0, 6))
        dem = (dem if case % 2 == 0 else dem.T).astype(np.float32)
        mask = (rng.random((8, 8)) < 0.35).astype(np.uint8)
        params = dict(mu=float(rng.uniform(0, 0.5)), xi=[INF, 500.0, 3000.0][case % 3],
                      flow_height=float(rng.uniform(0.5, 3)), persistence=float(rng.uniform(0, 1)),
                      randomness=float(rng.uniform(0, 0.6)), step_cells=[1.0, 0.5, 0.75][case % 3],
                      tan_alpha=[-1.0, 0.3][case % 2])
        both(avl, dem, mask, 5.0, params, 3, 40, int(rng.integers(0, 2**63)), case, f"8x8 case {case}")


def test_edge_cases(avl):
    dem = synth.alpine_dem(64, 500.0, seed=3)
    params = dict(mu=0.15, xi=1500.0, flow_height=1.0, persistence=0.9, randomness=0.16, step_cells=1.0,
                  tan_alpha=-1.0)
    empty = np.zeros((64, 64), np.uint8)
    got = gpu_run(avl, dem, empty, 10.0, params, 16, 100, 1)
    assert got[0].sum() == 0 and got[1].sum() == 0 and list(got[2]) == [0, 0, 0, 0]
    one = empty.copy()
    one[30, 31] = 1
    both(avl, dem, one, 10.0, params, 1, 500, 1, 0, "single particle")
    both(avl, dem, one, 10.0, params, 1000, 500, 1, 0, "one cell, 1000 replicas")   # many reservoir refills
    both(avl, dem, one, 10.0, params, 100, 0, 1, 0, "zero steps")
    full = np.ones((64, 64), np.uint8)
    both(avl, dem, full, 10.0, params, 3, 1, 5, 0, "one step everywhere")
    both(avl, dem, full, 10.0, params, 1, 300, 5, 0, "every cell")
    # one-row and one-column grids (the trajectory pass needs no 2x2 neighbourhood)
    line = (np.arange(40, dtype=np.float32)[::-1] * 7.0)[None, :].copy()
    both(avl, line, np.ones_like(line, np.uint8), 10.0, params, 5, 100, 2, 0, "1 x 40")
    both(avl, line.T.copy(), np.ones((40, 1), np.uint8), 10.0, params, 5, 100, 2, 0, "40 x 1")
    # step limit reached by every particle, and different seeds / run ids give different streams
    plane = synth.plane_dem(300, 80, 10.0, 35.0, 3000.0)
    top = np.zeros_like(plane, np.uint8)
    top[2:4, 35:45] = 1
    g1, _ = both(avl, plane, top, 10.0, dict(params, xi=INF), 9, 50, 11, 0, "limit")
    g2, _ = both(avl, plane, top, 10.0, dict(params, xi=INF), 9, 50, 11, 1, "limit run 1")
    assert g1[2][3] == 9 * 20
    assert not np.array_equal(g1[0], g2[0])


@pytest.mark.parametrize("scale", [1e-16, 1e-22, 1e-35])
def test_micro_relief(avl, scale):
    """Relief of ~scale metres: squared gradients fall below 2^-96 (and to subnormals), where the kernel's
    square root takes the compiler's full sequence for the wave instead of its short form."""
    rng = np.random.default_rng(int(-np.log10(scale)))
    dem = (rng.random((48, 40)) * scale).astype(np.float32)
    assert (dem > 0).all()
    mask = np.zeros(dem.shape, np.uint8)
    mask[::3, ::4] = 1
    params = dict(mu=0.0, xi=INF, randomness=0.2)
    got, ref = both(avl, dem, mask, 10.0, params, 7, 60, 3, 0, f"relief {scale}")
    assert ref.steps > 1000


@pytest.mark.parametrize("P", [2, 5, 63, 64, 65, 127, 4099])
def test_particles_per_cell_sweep(avl, P):
    """Slot decoding (release cell = slot / P, replica = slot mod P) for divisors around the 64-slot chunk
    size and a large prime."""
    dem = synth.alpine_dem(96, 700.0, seed=17)
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 28.0, 50.0, float(np.quantile(dem, 0.55)), INF)
    if P > 1000:  # keep the oracle short: a handful of cells
        sub = np.zeros(mask.size, np.uint8)
        sub[np.flatnonzero(mask)[::40]] = 1
        mask = sub.reshape(mask.shape)
    both(avl, dem, mask, 10.0, dict(mu=0.2, xi=2000.0, randomness=0.3), P, 300, 77, 5, f"P={P}")


def test_alpine_full_size(avl):
    """Full 2048^2 alpine tile at 256 particles per cell, in the launch shape the benchmark times: the whole
    pass against the oracle's whole pass (all host threads); then the GPU runs every 97th release cell, its
    complement and the whole mask, whose rasters must superpose."""
    from support import oracle_threads
    w = synth.make_workload("alpine")
    nrm = oracle.normals(w.dem, w.cell_size)
    mask = oracle.release_mask(nrm, w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    cells = np.flatnonzero(mask)
    assert 5e4 < len(cells) < 2e5
    sample = np.zeros(mask.size, np.uint8)
    sample[cells[::97]] = 1
    sample = sample.reshape(mask.shape)
    rest = (mask & (1 - sample)).astype(np.uint8)
    got_s, ref = both(avl, w.dem, sample, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed, 0,
                      "alpine sample")
    got_r = gpu_run(avl, w.dem, rest, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    got_f = gpu_run(avl, w.dem, mask, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    counts, vmax, stats = oracle_threads.full_pass(w.dem, mask, w.cell_size, w.params, w.particles_per_cell,
                                                   w.step_limit, w.seed)
    assert np.array_equal(got_f[0], counts)
    np.testing.assert_allclose(got_f[1], vmax, rtol=1e-5, atol=0)
    assert list(got_f[2]) == stats
    assert np.array_equal(got_f[0], got_s[0] + got_r[0])
    assert np.array_equal(got_f[1], np.maximum(got_s[1], got_r[1]))
    assert np.array_equal(got_f[2], got_s[2] + got_r[2])


def test_large_region_full_size(avl):
    """Full 8192^2 region at 5 m (256 MB DEM, ~1.4e6 release cells, 64 particles per cell, step limit 8000) in
    the benchmark's launch shape: the whole pass against the oracle's whole pass (run on all host threads),
    counts and statistics bit for bit, speeds within 1e-5; and the superposition of a 1-in-64 sample of the
    release cells and its complement equal to the whole pass."""
    from support import oracle_threads
    w = synth.make_workload("large")
    nrm = oracle.normals(w.dem, w.cell_size)
    mask = oracle.release_mask(nrm, w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    del nrm
    cells = np.flatnonzero(mask)
    assert 5e5 < len(cells) < 3e6
    got_f = gpu_run(avl, w.dem, mask, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    print(f"large region: {len(cells)} release cells, oracle on {oracle_threads.host_threads()} threads", flush=True)
    counts, vmax, stats = oracle_threads.full_pass(w.dem, mask, w.cell_size, w.params, w.particles_per_cell,
                                                   w.step_limit, w.seed)
    assert np.array_equal(got_f[0], counts)
    np.testing.assert_allclose(got_f[1], vmax, rtol=1e-5, atol=0)
    assert list(got_f[2]) == stats
    del counts, vmax
    sample = np.zeros(mask.size, np.uint8)
    sample[cells[::64]] = 1
    sample = sample.reshape(mask.shape)
    rest = (mask & (1 - sample)).astype(np.uint8)
    got_s = gpu_run(avl, w.dem, sample, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    got_r = gpu_run(avl, w.dem, rest, w.cell_size, w.params, w.particles_per_cell, w.step_limit, w.seed)
    assert np.array_equal(got_f[0], got_s[0] + got_r[0])
    assert np.array_equal(got_f[1], np.maximum(got_s[1], got_r[1]))
    assert np.array_equal(got_f[2], got_s[2] + got_r[2])


def test_tail_probe_times_every_block_and_leaves_the_pass_unchanged(avl):
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, w.cell_size), w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min,
                               w.z_max)
    plain = gpu_run(avl, w.dem, mask, w.cell_size, w.params, 8, 600, w.seed)
    grid = max(avl.trajectory_grid(v) for v in range(avl.tuning_variants()))
    buf = torch.zeros(3 * grid, dtype=torch.uint64, device="cuda")
    avl.set_probe(buf)
    try:
        got = gpu_run(avl, w.dem, mask, w.cell_size, w.params, 8, 600, w.seed)
    finally:
        avl.set_probe(None)
    for a, b in zip(got, plain):
        assert np.array_equal(a, b)
    t = host(buf).view(np.int64).reshape(-1, 3)
    t = t[t[:, 0] > 0]
    assert t.shape[0] > 0
    assert (t[:, 2] >= t[:, 0]).all()
    dry = t[t[:, 1] > 0]
    assert dry.shape[0] > 0 and (dry[:, 1] >= dry[:, 0]).all() and (dry[:, 2] >= dry[:, 1]).all()
