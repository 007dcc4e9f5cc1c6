"""GPU parity of the release texture at a finer resolution than the DEM (mult x mult texels per DEM cell):
the fine release map and the trajectory pass from it, through the C ABI, against the CPU oracle.

Bar: release map, hit counts, visited set and statistics bit-exact; max velocity within 1e-5 relative
(same binary32 arithmetic, expected exact). Ragged grids (not multiples of the kernel's four-texel
groups), several multipliers, an empty texture, a user-drawn texture (a release area given as a texture
rather than computed from the terrain), and mult = 1 against the plain entry points.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

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


def terrain(n=70, w=None, seed=31, relief=900.0):
    dem = synth.alpine_dem(n, relief, seed=seed)
    if w is not None:
        dem = np.ascontiguousarray(dem[:, :w])
    return dem


@pytest.mark.parametrize("shape", [(70, 70), (61, 53), (9, 7)])
@pytest.mark.parametrize("mult", [1, 2, 3, 4, 7])
def test_fine_release_map_bit_exact(avl, shape, mult):
    h, w = shape
    dem = terrain(max(h, w), seed=31 + mult)[:h, :w].copy()
    cs = 10.0
    nrm_ref = oracle.normals(dem, cs)
    zmin = float(np.quantile(dem, 0.5))
    ref = oracle.release_mask_fine(nrm_ref, dem, mult, 28.0, 46.0, zmin, 1e9)
    nrm = avl.normals(dev(dem), cs)
    got = host(avl.release_mask_fine(nrm, dev(dem), mult, 28.0, 46.0, zmin, 1e9))
    assert got.shape == (h * mult, w * mult)
    assert np.array_equal(got, ref), f"differ at {np.argwhere(got != ref)[:5]}"
    if mult == 1:
        assert np.array_equal(got, host(avl.release_mask(nrm, dev(dem), 28.0, 46.0, zmin, 1e9)))


def run_both(avl, dem, mask, mult, cs, params, P, S, seed, run=0):
    ref = oracle.trajectories_fine(dem, mask, mult, cs, oracle.make_params(**params), P, S, seed, run)
    res = avl.trajectories_fine(dev(dem), dev(mask), mult, cs, avl.Params.make(**params), P, S, seed, run)
    counts, vmax, stats = host(res.counts), host(res.vmax), host(res.stats)
    assert np.array_equal(counts, ref.counts), f"counts differ at {np.argwhere(counts != ref.counts)[:5]}"
    np.testing.assert_allclose(vmax, ref.vmax, rtol=VMAX_RTOL, atol=0)
    assert list(stats) == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit]
    return counts, vmax, stats


@pytest.mark.parametrize("mult,P", [(2, 16), (3, 8), (4, 4)])
def test_fine_trajectories_bit_exact(avl, mult, P):
    # 180 x 163 cells, 20-60 thousand release texels, 0.2-0.5 million particles
    dem = terrain(180, w=163, seed=40 + mult, relief=700.0)
    cs = 10.0
    nrm = oracle.normals(dem, cs)
    mask = oracle.release_mask_fine(nrm, dem, mult, 28.0, 50.0, float(np.quantile(dem, 0.4)), 1e9)
    assert mask.sum() > 10000
    counts, _, stats = run_both(avl, dem, mask, mult, cs, dict(mu=0.22, xi=1500.0), P, 600, seed=77, run=3)
    assert stats[0] > 500000 and counts.sum() > 0


def test_fine_mult_one_is_the_plain_pass(avl):
    dem = terrain(48, seed=5)
    cs = 10.0
    mask = oracle.release_mask(oracle.normals(dem, cs), dem, 25.0, 50.0, float(np.quantile(dem, 0.5)), 1e9)
    p = avl.Params.make(mu=0.2, xi=2000.0)
    a = avl.trajectories(dev(dem), dev(mask), cs, p, 4, 400, 11, 1)
    b = avl.trajectories_fine(dev(dem), dev(mask), 1, cs, p, 4, 400, 11, 1)
    assert np.array_equal(host(a.counts), host(b.counts))
    assert np.array_equal(host(a.vmax), host(b.vmax))
    assert np.array_equal(host(a.stats), host(b.stats))


def test_fine_user_texture_and_empty(avl):
    # a release area drawn by hand (a disc and a strip), as for a known event, at 5 texels per cell edge
    dem = terrain(40, seed=9)
    mult, cs = 5, 10.0
    hf, wf = 40 * mult, 40 * mult
    yy, xx = np.mgrid[0:hf, 0:wf]
    mask = (((yy - 60) ** 2 + (xx - 90) ** 2) < 15 ** 2) | ((yy >= 140) & (yy < 143) & (xx > 20) & (xx < 170))
    run_both(avl, dem, mask.astype(np.uint8), mult, cs, dict(mu=0.25, xi=1800.0), 2, 500, seed=5)
    counts, vmax, stats = run_both(avl, dem, np.zeros((hf, wf), np.uint8), mult, cs, dict(), 4, 100, seed=1)
    assert counts.sum() == 0 and vmax.max() == 0 and stats.sum() == 0


def test_fine_largest_multiplier(avl):
    # 16 x 16 texels per DEM cell (the maximum) on a small ragged tile, a sparse texture
    dem = terrain(24, w=19, seed=12, relief=400.0)[:21].copy()
    mult, cs = 16, 10.0
    nrm = oracle.normals(dem, cs)
    ref_map = oracle.release_mask_fine(nrm, dem, mult, 20.0, 60.0, float(np.quantile(dem, 0.3)), 1e9)
    got_map = host(avl.release_mask_fine(avl.normals(dev(dem), cs), dev(dem), mult, 20.0, 60.0,
                                         float(np.quantile(dem, 0.3)), 1e9))
    assert np.array_equal(got_map, ref_map)
    sparse = np.zeros_like(ref_map)
    sparse[::4, ::3] = ref_map[::4, ::3]
    assert sparse.sum() > 100
    run_both(avl, dem, sparse, mult, cs, dict(mu=0.2, xi=2000.0), 3, 400, seed=9)


def test_fine_alpine_full_size_sampled(avl):
    """The benchmark's fine-release leg: the 2048^2 alpine tile at 2 x 2 release texels per cell and 64
    particles per texel. The oracle runs every 389th release texel; the GPU runs that sample, its
    complement and the whole texture, whose rasters must be the sum (counts, statistics) and the maximum
    (speeds) of the two parts."""
    w = synth.make_workload("alpine")
    mult, P = 2, 64
    nrm = oracle.normals(w.dem, w.cell_size)
    fine = oracle.release_mask_fine(nrm, w.dem, mult, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max)
    del nrm
    got_map = host(avl.release_mask_fine(avl.normals(dev(w.dem), w.cell_size), dev(w.dem), mult, w.slope_min_deg,
                                         w.slope_max_deg, w.z_min, w.z_max))
    assert np.array_equal(got_map, fine)
    texels = np.flatnonzero(fine)
    assert 2e5 < len(texels) < 8e5
    sample = np.zeros(fine.size, np.uint8)
    sample[texels[::389]] = 1
    sample = sample.reshape(fine.shape)
    rest = (fine & (1 - sample)).astype(np.uint8)
    got_s = run_both(avl, w.dem, sample, mult, w.cell_size, w.params, P, w.step_limit, w.seed)
    p = avl.Params.make(**w.params)

    def gpu(m):
        r = avl.trajectories_fine(dev(w.dem), dev(m), mult, w.cell_size, p, P, w.step_limit, w.seed)
        return host(r.counts), host(r.vmax), host(r.stats)

    got_r = gpu(rest)
    got_f = gpu(fine)
    assert np.array_equal(got_f[0], got_s[0] + got_r[0])
    assert np.array_equal(got_f[1], np.maximum(got_s[1], got_r[1]))
    assert np.array_equal(got_f[2], got_s[2] + got_r[2])
