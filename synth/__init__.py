"""Seeded synthetic inputs: terrain rasters (DEMs), release scenarios and parameter sets.

The paper's datasets (the 501x151 *parabola* slope and the >100 km^2 Tyrol region, section 5.2) are not
available, so these generators stand in for them with the shapes of alpine workloads: 5-10 m cells
(section 5.2 recommends five to ten metres for avalanche runs) and square regions up to 8192^2 texels
(the texture limit of section 3).

This module holds no arithmetic of the avalanche method itself: it only makes inputs. Both the
HIP path and the CPU oracle consume what it returns. Every generator is deterministic in its seed
(numpy PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "diamond_square", "incline_fillet_dem", "alpine_dem", "plane_dem", "plane_to_flat_dem", "cone_dem",
    "nearest_rank", "bfs_blob", "param_sets", "Workload", "WORKLOADS", "make_workload",
]


# --------------------------------------------------------------------------------------------- fractals

def diamond_square(levels: int, hurst: float, rng: np.random.Generator) -> np.ndarray:
    """Midpoint-displacement (diamond-square) fBm on a (2^levels + 1)^2 grid, float64.

    The displacement standard deviation is multiplied by 2^-hurst at every halving of the step, so
    the surface has Hurst exponent ``hurst``. Edge points of the square step average their three
    in-grid neighbours.
    """
    n = (1 << levels) + 1
    z = np.zeros((n, n), dtype=np.float64)
    z[0, 0], z[0, -1], z[-1, 0], z[-1, -1] = rng.standard_normal(4)
    step = n - 1
    sigma = 1.0
    while step > 1:
        half = step // 2
        sigma *= 2.0 ** (-hurst)
        # diamond: square centres from the four corners
        a = z[0:n - 1:step, 0:n - 1:step]
        b = z[0:n - 1:step, step::step]
        c = z[step::step, 0:n - 1:step]
        d = z[step::step, step::step]
        z[half::step, half::step] = 0.25 * (a + b + c + d) + sigma * rng.standard_normal(a.shape)
        # square: edge midpoints from their (up to) four axis neighbours at distance `half`
        zp = np.pad(z, half, mode="constant", constant_values=np.nan)
        for r0, c0 in ((0, half), (half, 0)):
            nr = (n - 1 - r0) // step + 1
            nc = (n - 1 - c0) // step + 1

            def grab(dr: int, dc: int) -> np.ndarray:
                rs = r0 + half + dr
                cs = c0 + half + dc
                return zp[rs:rs + step * (nr - 1) + 1:step, cs:cs + step * (nc - 1) + 1:step]

            nb = np.stack([grab(-half, 0), grab(half, 0), grab(0, -half), grab(0, half)])
            cnt = np.sum(~np.isnan(nb), axis=0)
            mean = np.nansum(nb, axis=0) / cnt
            z[r0::step, c0::step] = mean + sigma * rng.standard_normal(mean.shape)
        step = half
    return z


def _levels_for(size: int) -> int:
    levels = max(1, math.ceil(math.log2(max(size, 2))))
    return levels


# --------------------------------------------------------------------------------------------- DEMs

def incline_fillet_dem(size: int = 256, cell_size: float = 10.0, slope_deg: float = 35.0,
                       kink_row: int = 160, noise_m: float = 5.0, hurst: float = 0.8, seed: int = 1) -> np.ndarray:
    """Inclined plane that blends into a flat runout, plus fBm noise.

    Height falls along +row (the y axis): z = tan(slope) * cs * (kink_row - r) down to row kink_row - 8,
    then a C^1 quadratic fillet tan(slope) * cs * (kink_row + 8 - r)^2 / 32 until row kink_row + 8, then
    0. Noise is diamond-square fBm cropped to the grid, shifted to zero mean and scaled to max |n| =
    ``noise_m`` metres. Returns float32 (size, size).
    """
    rng = np.random.default_rng(seed)
    k = math.tan(math.radians(slope_deg)) * cell_size
    r = np.arange(size, dtype=np.float64)[:, None]
    a, b = kink_row - 8, kink_row + 8
    base = np.where(r <= a, k * (kink_row - r), np.where(r < b, k * (b - r) ** 2 / 32.0, 0.0))
    noise = diamond_square(_levels_for(size), hurst, rng)[:size, :size]
    noise = noise - noise.mean()
    noise *= noise_m / np.abs(noise).max()
    return (base + noise).astype(np.float32)


def alpine_dem(size: int = 2048, relief_m: float = 2000.0, hurst: float = 0.8, seed: int = 2) -> np.ndarray:
    """Alpine-like fractal DEM: diamond-square fBm, normalised to [-1, 1], abs-folded into ridges
    (1 - |n|), rescaled to [0, relief_m]. Returns float32 (size, size)."""
    rng = np.random.default_rng(seed)
    z = diamond_square(_levels_for(size), hurst, rng)[:size, :size]
    lo, hi = z.min(), z.max()
    nrm = 2.0 * (z - lo) / (hi - lo) - 1.0
    ridge = 1.0 - np.abs(nrm)
    lo, hi = ridge.min(), ridge.max()
    return (relief_m * (ridge - lo) / (hi - lo)).astype(np.float32)


def plane_dem(h: int, w: int, cell_size: float, slope_deg: float, z0: float = 0.0) -> np.ndarray:
    """Exact inclined plane falling along +row: z[r][c] = z0 - tan(slope) * cs * r (float32)."""
    k = math.tan(math.radians(slope_deg)) * cell_size
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(z0 - k * r, (h, w)).astype(np.float32)


def plane_to_flat_dem(h: int, w: int, cell_size: float, slope_deg: float, kink_row: int) -> np.ndarray:
    """Plane falling along +row down to height 0 at ``kink_row``, flat (0) beyond (float32)."""
    k = math.tan(math.radians(slope_deg)) * cell_size
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(np.maximum(k * (kink_row - r), 0.0), (h, w)).astype(np.float32)


def cone_dem(n: int, cell_size: float, slope_deg: float, z0: float) -> np.ndarray:
    """Cone with apex at the centre cell of an n x n grid (n odd), falling with the given slope,
    floored at 0 (float32)."""
    k = math.tan(math.radians(slope_deg)) * cell_size
    c = (n - 1) / 2.0
    r = np.arange(n, dtype=np.float64)
    d = np.sqrt((r[:, None] - c) ** 2 + (r[None, :] - c) ** 2)
    return np.maximum(z0 - k * d, 0.0).astype(np.float32)


# --------------------------------------------------------------------------------------------- scenarios

def nearest_rank(z: np.ndarray, q: float) -> float:
    """Nearest-rank quantile: sorted(z)[floor(q * N)] (clamped to the last element)."""
    flat = np.sort(np.asarray(z, dtype=np.float32).ravel())
    i = min(int(math.floor(q * flat.size)), flat.size - 1)
    return float(flat[i])


def bfs_blob(eligible: np.ndarray, n_cells: int, seed: int) -> np.ndarray:
    """Connected release scenario: breadth-first growth (4-neighbourhood) over ``eligible`` cells from a
    seeded eligible start, until ``n_cells`` cells or the component is exhausted. Returns uint8 mask."""
    rng = np.random.default_rng(seed)
    h, w = eligible.shape
    cand = np.flatnonzero(eligible.ravel())
    out = np.zeros(h * w, dtype=np.uint8)
    if cand.size == 0 or n_cells <= 0:
        return out.reshape(h, w)
    start = int(cand[rng.integers(cand.size)])
    flat_ok = eligible.ravel().astype(bool)
    seen = np.zeros(h * w, dtype=bool)
    seen[start] = True
    frontier = [start]
    taken = 0
    while frontier and taken < n_cells:
        nxt = []
        for p in frontier:
            if taken >= n_cells:
                break
            out[p] = 1
            taken += 1
            r, c = divmod(p, w)
            for rr, cc in ((r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)):
                if 0 <= rr < h and 0 <= cc < w:
                    q = rr * w + cc
                    if flat_ok[q] and not seen[q]:
                        seen[q] = True
                        nxt.append(q)
        frontier = nxt
    return out.reshape(h, w)


def param_sets(n: int, seed: int) -> np.ndarray:
    """Friction parameter sets for ensemble sweeps: mu ~ U[0.1, 0.4], xi ~ U[500, 3000] m/s^2, flow
    height ~ U[0.5, 3] m. Returns float32 (n, 3) columns (mu, xi, h)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.1, 0.4, n)
    xi = rng.uniform(500.0, 3000.0, n)
    h = rng.uniform(0.5, 3.0, n)
    return np.stack([mu, xi, h], axis=1).astype(np.float32)


# --------------------------------------------------------------------------------------------- workloads

@dataclass
class Workload:
    """One named synthetic workload: DEM, cell size, release rule and model parameters."""
    name: str
    dem: np.ndarray
    cell_size: float
    slope_min_deg: float
    slope_max_deg: float
    z_min: float
    z_max: float
    particles_per_cell: int
    step_limit: int
    params: dict = field(default_factory=dict)
    seed: int = 1


DEFAULT_PARAMS = dict(mu=0.2, xi=2000.0, flow_height=1.0, persistence=0.9, randomness=0.16,
                      step_cells=1.0, tan_alpha=-1.0)

WORKLOADS = ("tiny", "alpine", "large")
LARGE_Q = 0.7


def make_workload(name: str) -> Workload:
    """The single-DEM plain-forward workloads.

    * ``tiny``:   256^2 incline (35 deg) + fillet + 5 m fBm at 10 m cells; release 30-45 deg above the
      70th elevation percentile; 16 particles/cell; mu 0.25, xi 1500, h 1; 2000 steps.
    * ``alpine``: 2048^2 ridged diamond-square fBm (Hurst 0.8, 2000 m relief) at 10 m; release 30-45 deg
      above the 93rd elevation percentile (the 70th gives ~4e5 cells on this surface; the 93rd gives
      the intended ~1e5); 256 particles/cell; mu 0.2, xi 2000, h 1; 4000 steps.
    * ``large``:  8192^2 ridged fBm (2500 m relief) at 5 m; 30-45 deg above ``large_q``; 64
      particles/cell; mu 0.2, xi 2000, h 1; 8000 steps.
    """
    inf = float("inf")
    if name == "tiny":
        dem = incline_fillet_dem(256, 10.0, seed=1)
        p = dict(DEFAULT_PARAMS, mu=0.25, xi=1500.0)
        return Workload(name, dem, 10.0, 30.0, 45.0, nearest_rank(dem, 0.7), inf, 16, 2000, p, seed=1)
    if name == "alpine":
        dem = alpine_dem(2048, 2000.0, seed=2)
        p = dict(DEFAULT_PARAMS)
        return Workload(name, dem, 10.0, 30.0, 45.0, nearest_rank(dem, 0.93), inf, 256, 4000, p, seed=2)
    if name == "large":
        dem = alpine_dem(8192, 2500.0, seed=3)
        p = dict(DEFAULT_PARAMS)
        return Workload(name, dem, 5.0, 30.0, 45.0, nearest_rank(dem, LARGE_Q), inf, 64, 8000, p, seed=3)
    raise KeyError(name)


# --------------------------------------------------------------------------------------------- ensembles

@dataclass
class Ensemble:
    """Batched workload: DEM tiles, one release scenario per tile, parameter sets and the run table
    (tile, scenario, param, run_id, seed) crossing every scenario with every parameter set."""
    dems: np.ndarray          # (n_tiles, H, W) float32
    masks: np.ndarray         # (n_masks, H, W) uint8
    params: list              # dicts of model parameters
    runs: list                # (tile, scenario, param, run_id, seed)
    cell_size: float
    particles_per_cell: int
    step_limit: int


def slope_deg(dem: np.ndarray, cell_size: float) -> np.ndarray:
    """Terrain slope in degrees from numpy.gradient (float64), for choosing scenario cells."""
    gy, gx = np.gradient(dem.astype(np.float64), cell_size)
    return np.degrees(np.arctan(np.hypot(gx, gy)))


def grow_region(score: np.ndarray, n_cells: int, start: int) -> np.ndarray:
    """Connected region of n_cells cells (4-neighbourhood) grown best-first from `start`: the frontier
    cell with the highest score joins next. Returns a uint8 mask."""
    import heapq
    h, w = score.shape
    flat = score.ravel()
    out = np.zeros(h * w, dtype=np.uint8)
    seen = np.zeros(h * w, dtype=bool)
    heap = [(-float(flat[start]), start)]
    seen[start] = True
    taken = 0
    while heap and taken < n_cells:
        _, p = heapq.heappop(heap)
        out[p] = 1
        taken += 1
        r, c = divmod(p, w)
        for rr, cc in ((r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)):
            if 0 <= rr < h and 0 <= cc < w:
                q = rr * w + cc
                if not seen[q]:
                    seen[q] = True
                    heapq.heappush(heap, (-float(flat[q]), q))
    return out.reshape(h, w)


# A 1024^2 window of the 2048^2 alpine statistics: relief 2000 m x 2^-0.8 (Hurst 0.8).
TILE_RELIEF_M = 2000.0 * 0.5 ** 0.8


def make_ensemble(n_tiles: int = 16, size: int = 1024, n_params: int = 64, particles_per_cell: int = 32,
                  step_limit: int = 2000, relief_m: float = TILE_RELIEF_M, cell_size: float = 10.0,
                  min_cells: int = 100, max_cells: int = 50000, seed: int = 12345) -> Ensemble:
    """The ensemble sweep: n_tiles ridged-fBm tiles (seeds 100, 101, ...; relief 1149 m, the alpine tile's
    statistics on a 1024^2 window), each with one connected release
    scenario of round(exp(U(ln min_cells, ln max_cells))) cells (sizes from seed 7): grown best-first
    (closest to 37.5 degrees first) from a seeded start cell of 30-45 degrees in the upper half of the
    elevations; crossed with n_params parameter sets mu ~ U[0.1, 0.4], xi ~ U[500, 3000], h ~ U[0.5, 3]
    (seed 8); persistence 0.9, randomness 0.16."""
    dems = np.stack([alpine_dem(size, relief_m, seed=100 + t) for t in range(n_tiles)])
    rng = np.random.default_rng(7)
    sizes = np.rint(np.exp(rng.uniform(math.log(min_cells), math.log(max_cells), n_tiles))).astype(int)
    masks = []
    for t in range(n_tiles):
        sl = slope_deg(dems[t], cell_size)
        cand = np.flatnonzero(((sl >= 30.0) & (sl <= 45.0) & (dems[t] >= np.median(dems[t]))).ravel())
        start = int(cand[np.random.default_rng(1000 + t).integers(cand.size)])
        masks.append(grow_region(-np.abs(sl - 37.5), int(sizes[t]), start))
    masks = np.stack(masks)
    ps = param_sets(n_params, 8)
    params = [dict(DEFAULT_PARAMS, mu=float(m), xi=float(x), flow_height=float(h)) for m, x, h in ps]
    runs = [(t, t, p, t * n_params + p, seed) for t in range(n_tiles) for p in range(n_params)]
    return Ensemble(dems, masks, params, runs, cell_size, particles_per_cell, step_limit)


@dataclass
class Calibration:
    """Differentiable-calibration workload: DEM, one connected release scenario with mass 1 per cell,
    the hidden (mu*, xi*) that makes the target deposit, and the starting point (mu0, xi0)."""
    dem: np.ndarray
    mask: np.ndarray
    mass: np.ndarray
    cell_size: float
    particles_per_cell: int
    step_limit: int
    mu_star: float
    xi_star: float
    mu0: float
    xi0: float
    flow_height: float
    seed: int


def make_calibration(size: int = 1024, n_cells: int = 5000, particles_per_cell: int = 128, step_limit: int = 3000,
                     relief_m: float = TILE_RELIEF_M, seed: int = 4) -> Calibration:
    """1024^2 ridged fBm DEM at 10 m (seed 4, relief 1149 m) with a 5000-cell release scenario grown best-first from a
    seeded steep start in the upper half of the elevations; mass 1 per release cell; target from
    mu* = 0.22, xi* = 1800; gradient taken at (mu0, xi0) = (0.26, 1400); h = 1 m."""
    dem = alpine_dem(size, relief_m, seed=seed)
    sl = slope_deg(dem, 10.0)
    cand = np.flatnonzero(((sl >= 30.0) & (sl <= 45.0) & (dem >= np.median(dem))).ravel())
    start = int(cand[np.random.default_rng(seed).integers(cand.size)])
    mask = grow_region(-np.abs(sl - 37.5), n_cells, start)
    mass = mask.astype(np.float32)
    return Calibration(dem, mask, mass, 10.0, particles_per_cell, step_limit, 0.22, 1800.0, 0.26, 1400.0, 1.0, seed)
