"""GPU checks of the memory microbenchmarks: replaying a recorded pass's raster atomics without aggregation
gives exactly the pass's counts and maxima; the gather replay reads exactly the texels the pass reads (the
XOR of their bits against the host's); the stream copy copies."""
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


@pytest.mark.parametrize("name,kw,S", [("tiny", {}, 2000), ("angle", dict(mu=0.05, xi=1200.0, tan_alpha=0.45), 2000),
                                       ("limit", dict(mu=0.01, xi=float("inf")), 45)])
def test_replays_reproduce_the_pass(avl, name, kw, S):
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, w.cell_size), w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min,
                               w.z_max)
    d, m = torch.from_numpy(w.dem).cuda(), torch.from_numpy(mask).cuda()
    p = avl.Params.make(**dict(w.params, **kw))
    print(f"membench replay case {name}: S={S}", flush=True)
    paths = avl.trajectory_paths(d, m, w.cell_size, p, 8, S, w.seed)
    counts, bits = avl.bench_atomics(w.dem.shape, paths)
    chk = avl.bench_gather(d, paths)
    torch.cuda.synchronize()
    assert torch.equal(counts.view(torch.int32), paths.run.counts.view(torch.int32))
    vmax = np.sqrt(bits.cpu().numpy().view(np.float32))
    assert np.array_equal(vmax, paths.run.vmax.cpu().numpy())
    ref = replay_ref.gather_checksum(w.dem, paths.points.cpu().numpy(), paths.ends.cpu().numpy(),
                                     paths.offsets.cpu().numpy())
    assert int(chk.item()) == ref


def test_stream_copy(avl):
    src = torch.arange(1 << 22, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    avl.bench_stream(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
