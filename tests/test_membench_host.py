"""Host checks of the memory microbenchmarks' replays, on paths built from oracle traces in the layout the
GPU records: every point, texel and raster cell the replay kernels index stays inside its buffer, and the
unaggregated atomic replay reproduces the oracle's own counts and maxima (so replaying a recorded pass
measures the pass's accumulation, nothing else)."""
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


def test_replay_indices_stay_inside_their_buffers():
    for kw, S in ((dict(mu=0.1, xi=1500.0), 300), (dict(mu=0.02, xi=float("inf")), 40),
                  (dict(mu=0.05, xi=1000.0, tan_alpha=0.4), 300)):
        dem, mask, p, S = _case(kw, S)
        H, W = dem.shape
        ends, pts, v2, off = replay_ref.paths_from_oracle(dem, mask, 10.0, p, 3, S, 9)
        assert off[-1] == pts.shape[0]
        idx = replay_ref.gather_points(ends, off)
        assert idx.min() >= 1 and idx.max() < pts.shape[0]
        o = replay_ref.gather_offsets(pts, idx, W)
        pad_bytes = (H + 2) * (W + 2) * 4
        assert o.min() >= 0 and (o + 4 * (W + 2) + 8).max() <= pad_bytes
        for k, e in enumerate(ends):  # the atomic replay's points: 0 .. steps, all inside the grid
            q = pts[int(off[k]):int(off[k]) + int(e >> 2) + 1]
            assert (q[:, 0] >= 0).all() and (q[:, 0] < W).all() and (q[:, 1] >= 0).all() and (q[:, 1] < H).all()


def test_atomic_replay_reproduces_the_oracle_rasters():
    for kw, S in ((dict(mu=0.1, xi=1500.0), 300), (dict(mu=0.05, xi=1000.0, tan_alpha=0.4), 300)):
        dem, mask, p, S = _case(kw, S)
        H, W = dem.shape
        ends, pts, v2, off = replay_ref.paths_from_oracle(dem, mask, 10.0, p, 3, S, 9)
        counts, vmax2 = replay_ref.atomic_replay(H, W, pts, v2, ends, off)
        ref = oracle.trajectories(dem, mask, 10.0, p, 3, S, 9)
        assert np.array_equal(counts, ref.counts)
        assert np.array_equal(np.sqrt(vmax2), ref.vmax)
