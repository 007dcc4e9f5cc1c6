"""Host references of the memory microbenchmarks (test support): the recorded-path layout the replays read,
built here from the oracle's traces; the wave-order schedule of a pass's gathers and cell visits; and what
each replay must produce."""
from __future__ import annotations

import numpy as np

import oracle


def paths_from_oracle(dem, mask, cs, params, P, S, seed, run=0):
    """(ends, points, speeds2, offsets) in the layout of the GPU's recorded paths, from oracle traces. A stopped
    particle's rejected target (which the traces do not keep) is stood in for by its last position."""
    cells = oracle.compact(mask)
    W = dem.shape[1]
    ends, pts, v2s, offs = [], [], [], [0]
    for cell in cells:
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


def _cell(p, W):
    return int(np.floor(p[1])) * W + int(np.floor(p[0]))


def schedule(ends, points, speeds2, offsets, W):
    """The wave-order schedule: per chunk of 64 consecutive particles, the t-th gather (visit) of every particle
    that has one, in particle order. Gathers are byte offsets of the 2 x 2 patch in the DEM padded by one
    texel; visits are (cell, bits of the largest v^2 of the steps that ended in it)."""
    gathers, visits = [], []
    n = len(ends)
    for c0 in range(0, n, 64):
        lanes = []
        for k in range(c0, min(n, c0 + 64)):
            e = int(ends[k])
            if e == 0xFFFFFFFF:
                lanes.append(([], []))
                continue
            steps, why, o = e >> 2, e & 3, int(offsets[k])
            g = []
            for t in range(steps + (1 if why == 2 else 0)):
                p = points[o + 1 + t]
                fr = int(np.floor(p[1] - np.float32(0.5))) + 1
                fc = int(np.floor(p[0] - np.float32(0.5))) + 1
                g.append((fr * (W + 2) + fc) * 4)
            v, at = [], 0
            while at <= steps:
                cell = _cell(points[o + at], W)
                cmax = np.float32(0.0) if at == 0 else speeds2[o + at]
                at += 1
                while at <= steps and _cell(points[o + at], W) == cell:
                    cmax = max(cmax, speeds2[o + at])
                    at += 1
                v.append((cell, int(np.float32(cmax).view(np.uint32))))
            lanes.append((g, v))
        for t in range(max((len(l[0]) for l in lanes), default=0)):
            gathers.extend(l[0][t] for l in lanes if t < len(l[0]))
        for t in range(max((len(l[1]) for l in lanes), default=0)):
            visits.extend(l[1][t] for l in lanes if t < len(l[1]))
    return np.array(gathers, np.uint32), np.array(visits, np.uint32).reshape(-1, 2)


def padded(dem):
    return np.pad(dem, 1, mode="edge").astype(np.float32)


def gather_checksum(dem, gathers):
    """XOR of the bits of every texel the gather replay reads."""
    W = dem.shape[1]
    bits = padded(dem).view(np.uint32).ravel()
    o = gathers.astype(np.int64) // 4
    acc = np.uint32(0)
    for part in (bits[o], bits[o + 1], bits[o + W + 2], bits[o + W + 3]):
        acc ^= np.bitwise_xor.reduce(part) if part.size else np.uint32(0)
    return int(acc)


def points_checksum(dem, points, ends, offsets):
    """The same XOR taken straight from the recorded points (every gather of every particle)."""
    W = dem.shape[1]
    idx = []
    for k, e in enumerate(ends):
        if e == 0xFFFFFFFF:
            continue
        n = int(e >> 2) + (1 if (e & 3) == 2 else 0)
        idx.append(np.arange(int(offsets[k]) + 1, int(offsets[k]) + 1 + n))
    idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    p = points[idx]
    fr = np.floor(p[:, 1] - np.float32(0.5)).astype(np.int64) + 1
    fc = np.floor(p[:, 0] - np.float32(0.5)).astype(np.int64) + 1
    return gather_checksum(dem, ((fr * (W + 2) + fc) * 4).astype(np.uint32))


def atomic_replay(H, W, visits):
    """Counts and per-cell max of v^2 that the atomic replay accumulates from the visits."""
    counts = np.zeros(H * W, np.uint32)
    bits = np.zeros(H * W, np.uint32)
    np.add.at(counts, visits[:, 0].astype(np.int64), 1)
    np.maximum.at(bits, visits[:, 0].astype(np.int64), visits[:, 1])
    return counts.reshape(H, W), bits.view(np.float32).reshape(H, W)
