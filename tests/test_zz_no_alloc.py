"""GPU test of the allocation-free trajectory entry point: through the C ABI it must give exactly what
avl_trajectories gives (same counts, speeds and statistics), on two calls in a row, the second on a smaller
grid, so that nothing left in the shared scratch by the first call leaks into the second."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _case(seed, h, w):
    rng = np.random.default_rng(seed)
    dem = synth.alpine_dem(size=max(h, w), relief_m=600.0, seed=seed)[:h, :w].astype(np.float32).copy()
    mask = np.zeros((h, w), np.uint8)
    mask[rng.random((h, w)) < 0.05] = 1
    return dem, mask


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_23364_amd as avl
    params = avl.Params.make(mu=0.2, xi=2000.0)
    for seed, (h, w), P in ((11, (300, 260), 16), (12, (97, 113), 8)):
        print(f"noalloc case seed={seed} shape={h}x{w} P={P}", flush=True)
        dem_np, mask_np = _case(seed, h, w)
        dem = torch.from_numpy(dem_np).cuda()
        mask = torch.from_numpy(mask_np).cuda()
        got = avl.trajectories_noalloc(dem, mask, 10.0, params, P, 1000, seed, 3)
        ref = avl.trajectories(dem, mask, 10.0, params, P, 1000, seed, 3)
        torch.cuda.synchronize()
        assert int(mask_np.sum()) > 0
        assert torch.equal(got.counts.view(torch.int32), ref.counts.view(torch.int32))
        assert torch.equal(got.vmax, ref.vmax)
        assert torch.equal(got.stats.view(torch.int64), ref.stats.view(torch.int64))
        assert int(got.stats[0].item()) > int(mask_np.sum()) * P  # particles moved
