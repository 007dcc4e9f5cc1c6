"""Host checks of the memory microbenchmarks, on paths built from oracle traces in the layout the GPU
records: every gather of the wave-order schedule and every raster cell it indexes stays inside its buffer,
the schedule holds every gather of the pass once, and the unaggregated atomic replay of its visits reproduces
the oracle's own counts and maxima (so replaying a recorded pass measures the pass's accumulation, nothing
else)."""
import numpy as np

import oracle
import synth
from support import replay_ref


def _case(kw, S):
    dem = synth.alpine_dem(64, 600.0, seed=17)[:45, :61].copy()
    nrm = oracle.normals(dem, 10.0)
    mask = oracle.release_mask(nrm, dem, 25.0, 50.0, float(np.quantile(dem, 0.6)), np.inf)
    p = oracle.make_params(**dict(synth.DEFAULT_PARAMS, **kw))
    return dem, mask, p, S


CASES = ((dict(mu=0.1, xi=1500.0), 300), (dict(mu=0.02, xi=float("inf")), 40),
         (dict(mu=0.05, xi=1000.0, tan_alpha=0.4), 300))


def test_schedule_stays_inside_its_buffers_and_holds_every_gather():
    for kw, S in CASES:
        dem, mask, p, S = _case(kw, S)
        H, W = dem.shape
        ends, pts, v2, off = replay_ref.paths_from_oracle(dem, mask, 10.0, p, 3, S, 9)
        assert off[-1] == pts.shape[0]
        g, v = replay_ref.schedule(ends, pts, v2, off, W)
        pad_bytes = (H + 2) * (W + 2) * 4
        assert g.astype(np.int64).min() >= 0 and (g.astype(np.int64) + 4 * (W + 2) + 8).max() <= pad_bytes
        assert v[:, 0].max() < H * W
        n_gathers = sum(int(e >> 2) + (1 if (e & 3) == 2 else 0) for e in ends)
        assert g.size == n_gathers
        assert replay_ref.gather_checksum(dem, g) == replay_ref.points_checksum(dem, pts, ends, off)


def test_atomic_replay_reproduces_the_oracle_rasters():
    for kw, S in CASES:
        dem, mask, p, S = _case(kw, S)
        H, W = dem.shape
        ends, pts, v2, off = replay_ref.paths_from_oracle(dem, mask, 10.0, p, 3, S, 9)
        _, v = replay_ref.schedule(ends, pts, v2, off, W)
        counts, vmax2 = replay_ref.atomic_replay(H, W, v)
        ref = oracle.trajectories(dem, mask, 10.0, p, 3, S, 9)
        assert np.array_equal(counts, ref.counts)
        assert np.array_equal(np.sqrt(vmax2), ref.vmax)
