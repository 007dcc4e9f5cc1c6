"""GPU parity of the overlay mipmap (avl_overlay_mipmap) against the oracle: bit-exact counts (uint64
sums) and speeds (maxima) on every level, for ragged, degenerate and full-size grids."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avl():
    import paper_2506_23364_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return m


def check(avl, c, v):
    pyr = avl.overlay_mipmap(torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
    torch.cuda.synchronize()
    ref = oracle.mipmap(c, v)
    assert len(pyr) == len(ref)
    for (gc, gv), (rc, rv) in zip(pyr, ref):
        assert np.array_equal(gc.cpu().numpy(), rc)
        assert np.array_equal(gv.cpu().numpy(), rv)


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (2, 3), (37, 53), (64, 64), (65, 65), (1000, 3),
                                   (129, 4097)])
def test_random_rasters(avl, shape):
    rng = np.random.default_rng(shape[0] * 7919 + shape[1])
    c = rng.integers(0, 1 << 31, shape).astype(np.uint32)  # coarse levels need the 64-bit sums
    v = (rng.random(shape) * (rng.random(shape) < 0.5) * 80).astype(np.float32)
    check(avl, c, v)


def test_alpine_overlay(avl):
    """The mipmap of the alpine tile's overlay (2048^2: 11 levels, two passes of the tiled kernel)."""
    w = synth.make_workload("alpine")
    dem = torch.from_numpy(w.dem).cuda()
    _, _, res = avl.overlay(dem, w.cell_size, w.slope_min_deg, w.slope_max_deg, w.z_min, w.z_max,
                            avl.Params.make(**w.params), 16, w.step_limit, w.seed)
    torch.cuda.synchronize()
    check(avl, res.counts.cpu().numpy(), res.vmax.cpu().numpy())
