"""Pins of the oracle's release texture at a finer resolution than the DEM (section 5.2: the user chooses
the texture resolution at which release points are evaluated, and known release points can come as a
texture of their own).

* release map: at one texel per DEM cell it is the plain release map; on normal and height fields that
  are linear along one axis the filtered values, and so the map, follow the closed form of the line
  (columns and rows separately, so a transposed index fails); on a random field it agrees with scipy's
  bilinear interpolant of the texel centres, clamped to the centre grid;
* particles: each starts at the centre ((C + 1/2) / m, (R + 1/2) / m) of its release texel; on an exact
  plane without randomness they run straight down the column of their DEM cell with the closed-form speed
  of the friction law; their random stream is keyed by the texel's index in the release texture (checked
  against rocRAND's Philox4x32-10 through the first direction); one texel per DEM cell gives the plain
  run; runs superpose over disjoint release textures.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from tests.support.philox_ref import philox_blocks

INF = float("inf")


def f32(v):
    return float(np.float32(v))


def normals_from(nz):
    """normals4 whose nz channel is `nz` (the release map reads only nz)."""
    h, w = nz.shape
    n4 = np.zeros((h, w, 4), np.float64)
    n4[..., 2] = nz
    return n4


def slope_bounds(nz_lo, nz_hi):
    """(smin, smax) in degrees whose cosines are nz_hi and nz_lo."""
    return math.degrees(math.acos(nz_hi)), math.degrees(math.acos(nz_lo))


# ------------------------------------------------------------------------------------------ release map

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fine_map_at_one_texel_per_cell_is_the_release_map(prec):
    dem = synth.alpine_dem(80, 900.0, seed=21)
    nrm = oracle.normals(dem, 10.0, prec=prec)
    zmin = float(np.quantile(dem, 0.4))
    plain = oracle.release_mask(nrm, dem, 28.0, 47.0, zmin, 1e9, prec=prec)
    fine = oracle.release_mask_fine(nrm, dem, 1, 28.0, 47.0, zmin, 1e9, prec=prec)
    assert plain.any() and not plain.all()
    np.testing.assert_array_equal(fine, plain)


def _centres(n, mult):
    """Exact centres (k + 1/2) / mult of the fine texels along an axis of n DEM cells."""
    return [Fraction(2 * k + 1, 2 * mult) for k in range(n * mult)]


def _line(n, a, b, mult):
    """Exact value of the filtered field a + b * (texel index) at each fine centre, clamped to the grid."""
    out = []
    for x in _centres(n, mult):
        t = min(max(x - Fraction(1, 2), Fraction(0)), Fraction(n - 1))
        out.append(Fraction(a) + Fraction(b) * t)
    return out


@pytest.mark.parametrize("axis", [1, 0])
@pytest.mark.parametrize("mult", [2, 3, 4])
def test_fine_map_follows_a_linear_nz_field(axis, mult):
    # nz = 1/2 + k/64 along one axis: the filtered nz at every fine centre is that line at the centre
    # (clamped to the first and last texel centre), so the steepness window selects a known interval
    h, w = (7, 11) if axis == 1 else (11, 7)
    n = w if axis == 1 else h
    k = np.arange(n, dtype=np.float64)
    line = 0.5 + k / 64.0
    nz = np.broadcast_to(line[None, :] if axis == 1 else line[:, None], (h, w))
    dem = np.zeros((h, w), np.float32)
    lo, hi = 0.5 + 2.3 / 64.0, 0.5 + 7.1 / 64.0
    smin, smax = slope_bounds(lo, hi)
    got = oracle.release_mask_fine(normals_from(nz), dem, mult, smin, smax, -1.0, 1.0, prec="f64")
    vals = _line(n, Fraction(1, 2), Fraction(1, 64), mult)
    cmin, cmax = math.cos(math.radians(smax)), math.cos(math.radians(smin))
    want1d = np.array([cmin <= float(v) <= cmax for v in vals], np.uint8)
    assert 0 < want1d.sum() < len(want1d)
    want = np.broadcast_to(want1d[None, :] if axis == 1 else want1d[:, None], got.shape)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("axis", [1, 0])
def test_fine_map_follows_a_linear_height_field(axis):
    # heights 3 m per texel along one axis, flat normals: the elevation window selects the fine texels
    # whose filtered height (the line at their centre) lies in it
    mult, h, w = 4, 9, 13
    n = w if axis == 1 else h
    line = 100.0 + 3.0 * np.arange(n, dtype=np.float64)
    dem = np.broadcast_to(line[None, :] if axis == 1 else line[:, None], (h, w)).astype(np.float32)
    nz = np.ones((h, w))
    zmin, zmax = 100.0 + 3.0 * 2.1, 100.0 + 3.0 * 5.6
    got = oracle.release_mask_fine(normals_from(nz), dem, mult, 0.0, 10.0, zmin, zmax, prec="f64")
    vals = _line(n, 100, 3, mult)
    want1d = np.array([zmin <= float(v) <= zmax for v in vals], np.uint8)
    assert 0 < want1d.sum() < len(want1d)
    want = np.broadcast_to(want1d[None, :] if axis == 1 else want1d[:, None], got.shape)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("mult", [2, 3, 5])
def test_fine_map_matches_scipy_bilinear(mult):
    rng = np.random.default_rng(5 + mult)
    h, w = 10, 14
    nz = 0.6 + 0.4 * rng.random((h, w))
    dem = (1000.0 * rng.random((h, w))).astype(np.float32)
    yc, xc = np.arange(h) + 0.5, np.arange(w) + 0.5
    fn = RegularGridInterpolator((yc, xc), nz)
    fz = RegularGridInterpolator((yc, xc), dem.astype(np.float64))
    smin, smax = slope_bounds(0.72, 0.9)
    zmin, zmax = 250.0, 800.0
    got = oracle.release_mask_fine(normals_from(nz), dem, mult, smin, smax, zmin, zmax, prec="f64")
    cmin, cmax = math.cos(math.radians(smax)), math.cos(math.radians(smin))
    R, C = np.meshgrid(np.arange(h * mult), np.arange(w * mult), indexing="ij")
    y = np.clip((R + 0.5) / mult, 0.5, h - 0.5)
    x = np.clip((C + 0.5) / mult, 0.5, w - 0.5)
    pts = np.stack([y.ravel(), x.ravel()], axis=1)
    nzi, zi = fn(pts).reshape(R.shape), fz(pts).reshape(R.shape)
    want = ((cmin <= nzi) & (nzi <= cmax) & (zmin <= zi) & (zi <= zmax)).astype(np.uint8)
    # texels whose filtered value sits within rounding of a bound may go either way
    near = ((np.abs(nzi - cmin) < 1e-12) | (np.abs(nzi - cmax) < 1e-12) | (np.abs(zi - zmin) < 1e-9)
            | (np.abs(zi - zmax) < 1e-9))
    assert want.sum() > 20 and (~near).sum() > 0.99 * near.size
    np.testing.assert_array_equal(got[~near], want[~near])


# ------------------------------------------------------------------------------------------ particles

def exact_plane(h, w, k=7.0):
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(k * h - k * r, (h, w)).astype(np.float32)


@pytest.mark.parametrize("mult", [1, 2, 3, 4])
def test_release_point_is_the_texel_centre(mult):
    dem = exact_plane(12, 10)
    p = oracle.make_params(mu=0.1, xi=INF, randomness=0.3)
    for tr, tc in ((0, 0), (5, 7), (12 * mult - 1, 10 * mult - 1), (3 * mult + 1, 2 * mult + mult - 1)):
        t = oracle.trace(dem, 10.0, p, r=tr, c=tc, replica=3, step_limit=0, seed=9, prec="f64", mult=mult)
        assert t.x[0] == float(Fraction(2 * tc + 1, 2 * mult))
        assert t.y[0] == float(Fraction(2 * tr + 1, 2 * mult))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mult", [2, 3])
def test_plane_column_closed_form(prec, mult):
    # exact plane falling 7 m per row, no randomness, no friction, no drag: every particle of texel (R, C)
    # runs straight down the column C // mult and leaves the grid at the bottom; it enters each row from
    # R // mult on once, arriving in row R // mult + n with v^2 = 2 g n * 7 m while it stays above the last
    # texel centre (below it the clamped patch is flat)
    h, w, cs, P = 14, 6, 10.0, 3
    dem = exact_plane(h, w)
    p = oracle.make_params(mu=0.0, xi=INF, persistence=0.9, randomness=0.0)
    R, C = 2 * mult + 1, 4 * mult + mult - 1
    mask = np.zeros((h * mult, w * mult), np.uint8)
    mask[R, C] = 1
    res = oracle.trajectories_fine(dem, mask, mult, cs, p, P, 100, seed=3, prec=prec)
    r0, c0 = R // mult, C // mult
    want = np.zeros((h, w), np.uint32)
    want[r0:, c0] = P
    np.testing.assert_array_equal(res.counts, want)
    assert (res.n_exit, res.n_stop, res.n_limit) == (P, 0, 0)
    assert res.steps == P * (h - r0)
    g = 9.81 if prec == "f64" else f32(9.81)
    y0 = (R + 0.5) / mult
    for n in range(1, h - r0):
        if y0 + n > h - 0.5:
            break
        v = math.sqrt(2.0 * g * n * 7.0)
        assert abs(float(res.vmax[r0 + n, c0]) - v) < 1e-6 * v
    assert res.vmax[r0, c0] == 0.0


def _uniforms(n, replica, word, run, seed):
    o = philox_blocks(np.array([[n >> 1, replica, word, run, seed & 0xFFFFFFFF, seed >> 32]], np.uint32))[0]
    ux, uy = (int(o[2]), int(o[3])) if n & 1 else (int(o[0]), int(o[1]))
    return 2.0 * (ux >> 8) * 2.0 ** -24 - 1.0, 2.0 * (uy >> 8) * 2.0 ** -24 - 1.0


@pytest.mark.parametrize("mult", [1, 2, 3])
def test_random_stream_is_keyed_by_the_release_texel(mult):
    # on a plane falling along +y with persistence 1 the first new direction is (0, 1) + rnd * (rx, ry)
    # normalised, with (rx, ry) the uniforms of counter (0, replica, R * mult * W + C, run)
    h, w = 16, 12
    dem = exact_plane(h, w)
    rnd, seed, run = 0.5, 0xFEDCBA9876543210, 6
    p = oracle.make_params(mu=0.0, xi=INF, persistence=1.0, randomness=rnd)
    seen = set()
    for R, C, j in ((3 * mult, 5 * mult, 0), (3 * mult + mult - 1, 5 * mult + 1, 0), (7 * mult, 2 * mult + 1, 4)):
        t = oracle.trace(dem, 10.0, p, r=R, c=C, replica=j, step_limit=2, seed=seed, run=run, prec="f64",
                         mult=mult)
        rx, ry = _uniforms(0, j, R * mult * w + C, run, seed)
        wx, wy = f32(rnd) * rx, 1.0 + f32(rnd) * ry
        wn = math.hypot(wx, wy)
        assert abs(t.rows[1, 5] - wx / wn) < 1e-12 and abs(t.rows[1, 6] - wy / wn) < 1e-12
        seen.add((round(t.rows[1, 5], 12), round(t.rows[1, 6], 12)))
    assert len(seen) == 3


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_one_texel_per_cell_is_the_plain_run(prec):
    dem = synth.alpine_dem(48, 700.0, seed=4)
    nrm = oracle.normals(dem, 10.0, prec=prec)
    mask = oracle.release_mask(nrm, dem, 25.0, 50.0, float(np.quantile(dem, 0.5)), 1e9, prec=prec)
    p = oracle.make_params(mu=0.25, xi=1500.0)
    a = oracle.trajectories(dem, mask, 10.0, p, 4, 300, seed=7, run=2, prec=prec)
    b = oracle.trajectories_fine(dem, mask, 1, 10.0, p, 4, 300, seed=7, run=2, prec=prec)
    np.testing.assert_array_equal(a.counts, b.counts)
    np.testing.assert_array_equal(a.vmax, b.vmax)
    assert (a.steps, a.n_exit, a.n_stop, a.n_limit) == (b.steps, b.n_exit, b.n_stop, b.n_limit)


def test_fine_runs_superpose():
    # counts add and speeds take the maximum over a split of the release texture into disjoint parts
    dem = synth.alpine_dem(32, 500.0, seed=8)
    mult = 3
    rng = np.random.default_rng(2)
    mask = (rng.random((32 * mult, 32 * mult)) < 0.02).astype(np.uint8)
    part = (rng.random(mask.shape) < 0.5).astype(np.uint8)
    p = oracle.make_params(mu=0.2, xi=2000.0)
    whole = oracle.trajectories_fine(dem, mask, mult, 10.0, p, 2, 200, seed=1)
    a = oracle.trajectories_fine(dem, mask * part, mult, 10.0, p, 2, 200, seed=1)
    b = oracle.trajectories_fine(dem, mask * (1 - part), mult, 10.0, p, 2, 200, seed=1)
    np.testing.assert_array_equal(whole.counts, a.counts + b.counts)
    np.testing.assert_array_equal(whole.vmax, np.maximum(a.vmax, b.vmax))
    assert whole.steps == a.steps + b.steps
