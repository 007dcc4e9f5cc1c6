"""Host references of the memory microbenchmarks' replays (test support): the recorded-path layout the
replays read, built here from the oracle's traces, and what each replay must produce on it."""
from __future__ import annotations

import numpy as np

import oracle


def paths_from_oracle(dem, mask, cs, params, P, S, seed, run=0):
    """(ends, points, speeds2, offsets) in the layout of the GPU's recorded paths, from oracle traces. A stopped
    particle's rejected target (which the traces do not keep) is stood in for by its last position."""
    cells = oracle.compact(mask)
    W = dem.shape[1]
    ends, pts, v2s, offs = [], [], [], [0]
    for i, cell in enumerate(cells):
        r, c = divmod(int(cell), W)
        for j in range(P):
            tr = oracle.trace(dem, cs, params, r, c, j, S, seed, run)
            steps = tr.rows.shape[0] - 1
            ends.append((steps << 2) | tr.reason)
            xy = np.stack([tr.x, tr.y], 1)
            v2 = tr.v2.copy()
            v2[0] = 0.0
            if tr.reason == 2:
                xy = np.concatenate([xy, xy[-1:]])
                v2 = np.concatenate([v2, [0.0]])
            pts.append(xy)
            v2s.append(v2)
            offs.append(offs[-1] + xy.shape[0])
    return (np.array(ends, np.uint32), np.concatenate(pts).astype(np.float32), np.concatenate(v2s).astype(np.float32),
            np.array(offs, np.uint64))


def gather_points(ends, offsets):
    """Indices of the points the gather replay reads: 1 .. steps (+ 1 for a stop) of each particle."""
    idx = []
    for k, e in enumerate(ends):
        if e == 0xFFFFFFFF:
            continue
        n = int(e >> 2) + (1 if (e & 3) == 2 else 0)
        idx.append(np.arange(int(offsets[k]) + 1, int(offsets[k]) + 1 + n))
    return np.concatenate(idx) if idx else np.zeros(0, np.int64)


def padded(dem):
    return np.pad(dem, 1, mode="edge").astype(np.float32)


def gather_offsets(points, idx, W):
    """Byte offsets into the padded DEM of the upper row of each gathered 2 x 2 patch."""
    p = points[idx]
    sx = p[:, 0] - np.float32(0.5)
    sy = p[:, 1] - np.float32(0.5)
    return ((np.floor(sy).astype(np.int64) + 1) * (W + 2) + np.floor(sx).astype(np.int64) + 1) * 4


def gather_checksum(dem, points, ends, offsets):
    """XOR of the bits of every texel the gather replay reads."""
    H, W = dem.shape
    bits = padded(dem).view(np.uint32).ravel()
    o = gather_offsets(points, gather_points(ends, offsets), W) // 4
    acc = np.uint32(0)
    for part in (bits[o], bits[o + 1], bits[o + W + 2], bits[o + W + 3]):
        acc ^= np.bitwise_xor.reduce(part) if part.size else np.uint32(0)
    return int(acc)


def atomic_replay(H, W, points, speeds2, ends, offsets):
    """Counts and per-cell max of v^2 that the atomic replay accumulates (one entry per cell entered, the
    maximum over the accepted steps that end in the cell)."""
    counts = np.zeros(H * W, np.uint32)
    vmax2 = np.zeros(H * W, np.float32)
    for k, e in enumerate(ends):
        if e == 0xFFFFFFFF:
            continue
        o, n = int(offsets[k]), int(e >> 2)
        p = points[o:o + n + 1]
        cell = np.floor(p[:, 1]).astype(np.int64) * W + np.floor(p[:, 0]).astype(np.int64)
        new = np.concatenate([[True], cell[1:] != cell[:-1]])
        np.add.at(counts, cell[new], 1)
        np.maximum.at(vmax2, cell[1:], speeds2[o + 1:o + n + 1])
    return counts.reshape(H, W), vmax2.reshape(H, W)
