"""GPU checks of the memory microbenchmarks: the GPU's wave-order schedule of a recorded pass equals the host's
on the same recorded paths; replaying its cell visits as unaggregated atomics gives exactly the pass's counts
and maxima; the gather replay reads exactly the pass's texels (the XOR of their bits against the host's); the
stream copy copies."""
import numpy as np
import pytest
import torch

import oracle
import synth
from support import replay_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avl():
    import paper_2506_23364_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return m


def _tiny():
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, w.cell_size), w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min,
                               w.z_max)
    return w, mask


def test_schedule_equals_the_host_schedule(avl):
    dem = synth.alpine_dem(96, 700.0, seed=33)[:70, :83].copy()
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 25.0, 50.0, float(np.quantile(dem, 0.7)), np.inf)
    d, m = torch.from_numpy(dem).cuda(), torch.from_numpy(mask).cuda()
    for kw, S in ((dict(mu=0.1, xi=1500.0), 400), (dict(mu=0.02, xi=float("inf")), 50),
                  (dict(mu=0.05, xi=1000.0, tan_alpha=0.4), 400)):
        print(f"membench schedule case {kw} S={S}", flush=True)
        p = avl.Params.make(**dict(synth.DEFAULT_PARAMS, **kw))
        paths = avl.trajectory_paths(d, m, 10.0, p, 5, S, 3)
        sched = avl.bench_schedule(dem.shape, paths)
        torch.cuda.synchronize()
        g, v = replay_ref.schedule(paths.ends.cpu().numpy(), paths.points.cpu().numpy(), paths.speeds2.cpu().numpy(),
                                   paths.offsets.cpu().numpy(), dem.shape[1])
        assert np.array_equal(sched.gathers.cpu().numpy(), g)
        assert np.array_equal(sched.visits.cpu().numpy(), v)


@pytest.mark.parametrize("name,kw,S", [("tiny", {}, 2000), ("angle", dict(mu=0.05, xi=1200.0, tan_alpha=0.45), 2000),
                                       ("limit", dict(mu=0.01, xi=float("inf")), 45)])
def test_replays_reproduce_the_pass(avl, name, kw, S):
    w, mask = _tiny()
    d, m = torch.from_numpy(w.dem).cuda(), torch.from_numpy(mask).cuda()
    p = avl.Params.make(**dict(w.params, **kw))
    print(f"membench replay case {name}: S={S}", flush=True)
    paths = avl.trajectory_paths(d, m, w.cell_size, p, 8, S, w.seed)
    sched = avl.bench_schedule(w.dem.shape, paths)
    counts, bits = avl.bench_atomics(w.dem.shape, sched)
    chk = avl.bench_gather(d, sched)
    torch.cuda.synchronize()
    assert torch.equal(counts.view(torch.int32), paths.run.counts.view(torch.int32))
    vmax = np.sqrt(bits.cpu().numpy().view(np.float32))
    assert np.array_equal(vmax, paths.run.vmax.cpu().numpy())
    ends = paths.ends.cpu().numpy()
    ref = replay_ref.points_checksum(w.dem, paths.points.cpu().numpy(), ends, paths.offsets.cpu().numpy())
    assert int(chk.item()) == ref
    assert sched.gathers.numel() == int(sum(int(e >> 2) + (1 if (e & 3) == 2 else 0) for e in ends))


def test_stream_copy(avl):
    src = torch.arange((1 << 22) + 12, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    avl.bench_stream(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
