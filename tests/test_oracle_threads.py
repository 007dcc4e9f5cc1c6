"""The threaded full-pass helper of the GPU tests equals the oracle's single call (the chunks of release cells
superpose exactly), so a full-size GPU check against it is a check against the oracle."""
import numpy as np

import oracle
import synth
from support import oracle_threads


def test_threaded_full_pass_equals_one_oracle_call():
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, w.cell_size), w.dem, w.slope_min_deg, w.slope_max_deg, w.z_min,
                               w.z_max)
    params = dict(w.params)
    counts, vmax, stats = oracle_threads.full_pass(w.dem, mask, w.cell_size, params, 4, 600, w.seed, 3, chunks=37)
    ref = oracle.trajectories(w.dem, mask, w.cell_size, oracle.make_params(**params), 4, 600, w.seed, 3)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(vmax, ref.vmax)
    assert stats == [ref.steps, ref.n_exit, ref.n_stop, ref.n_limit]


def test_run_all_keeps_job_order():
    assert oracle_threads.run_all(range(50), lambda k: k * k, threads=4) == [k * k for k in range(50)]
