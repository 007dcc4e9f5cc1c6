"""Full-size oracle runs on all host threads (test support): the oracle's C calls release the GIL, so a pool of
threads runs independent oracle calls side by side."""
from __future__ import annotations

import os
import queue
import threading

import numpy as np

import oracle


def host_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run_all(jobs, fn, threads: int | None = None):
    """fn(job) for every job, `threads` at a time; returns the results in job order (exceptions re-raised)."""
    jobs = list(jobs)
    out = [None] * len(jobs)
    errs = []
    todo = queue.Queue()
    for i, j in enumerate(jobs):
        todo.put((i, j))
    oracle._lib("f32")

    def worker():
        while True:
            try:
                i, j = todo.get_nowait()
            except queue.Empty:
                return
            try:
                out[i] = fn(j)
            except Exception as e:  # noqa: BLE001 - re-raised below
                errs.append(e)

    ts = [threading.Thread(target=worker) for _ in range(threads or host_threads())]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if errs:
        raise errs[0]
    return out


def full_pass(dem, mask, cs, params, P, S, seed, run=0, chunks: int = 64):
    """The oracle's whole pass over `mask`, split into chunks of consecutive release cells run side by side and
    merged exactly: (counts uint32, vmax float32, [steps, exits, stops, limit ends])."""
    cells = np.flatnonzero(mask)
    parts = [c for c in np.array_split(cells, chunks) if c.size]
    p = oracle.make_params(**params)

    def one(chunk):
        m = np.zeros(mask.size, np.uint8)
        m[chunk] = 1
        r = oracle.trajectories(dem, m.reshape(mask.shape), cs, p, P, S, seed, run)
        return r.counts, r.vmax, (r.steps, r.n_exit, r.n_stop, r.n_limit)

    counts = np.zeros(mask.shape, np.uint64)
    vmax = np.zeros(mask.shape, np.float32)
    stats = np.zeros(4, np.uint64)
    # merge in groups so that at most a few partial rasters are alive at once
    for g in range(0, len(parts), host_threads()):
        for c, v, s in run_all(parts[g:g + host_threads()], one):
            counts += c
            np.maximum(vmax, v, out=vmax)
            stats += np.array(s, np.uint64)
    return counts.astype(np.uint32), vmax, [int(v) for v in stats]
