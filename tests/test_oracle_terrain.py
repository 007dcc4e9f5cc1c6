"""Pins of the oracle's terrain passes: normals/steepness, release mask, release-cell compaction.

Section 5.2: the normals node computes surface normals per DEM texel; the release-point node keeps
texels whose steepness is within the user's range and outputs a binary map; particles are then
released per coded texel. The gradient is pinned bit-exactly to numpy.gradient (the textbook finite
difference), slopes to closed forms on planes and cones, compaction to numpy.flatnonzero.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _dems():
    rng = np.random.default_rng(5)
    yield "tiny", synth.incline_fillet_dem(256, 10.0, seed=1), 10.0
    yield "rand_ragged", (rng.standard_normal((37, 53)) * 30).astype(np.float32), 7.5
    yield "two_by_two", np.array([[0, 1], [3, 7]], np.float32), 2.0
    yield "alpine_crop", synth.alpine_dem(256, 800.0, seed=9), 5.0


@pytest.mark.parametrize("name,dem,cs", list(_dems()), ids=[d[0] for d in _dems()])
def test_gradient_matches_numpy_gradient(name, dem, cs):
    gy, gx = np.gradient(dem, np.float32(cs))
    assert gx.dtype == np.float32
    nrm = oracle.normals(dem, cs)
    l = np.sqrt((gx * gx + gy * gy) + np.float32(1))
    assert np.array_equal(nrm[..., 0], -(gx / l))
    assert np.array_equal(nrm[..., 1], -(gy / l))
    assert np.array_equal(nrm[..., 2], np.float32(1) / l)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_normals_unit_and_slope(prec):
    dem = synth.alpine_dem(128, 600.0, seed=4)
    nrm = oracle.normals(dem, 10.0, prec)
    norm = np.sqrt((nrm[..., :3].astype(np.float64) ** 2).sum(-1))
    tol = 4e-7 if prec == "f32" else 1e-15
    assert np.max(np.abs(norm - 1)) < tol
    # slope channel = angle between normal and vertical
    ang = np.degrees(np.arccos(np.clip(nrm[..., 2].astype(np.float64), -1, 1)))
    assert np.max(np.abs(ang - nrm[..., 3])) < (2e-3 if prec == "f32" else 1e-6)


@pytest.mark.parametrize("theta", [10.0, 30.0, 35.0, 44.9, 60.0])
def test_plane_slope_closed_form(theta):
    dem = synth.plane_dem(16, 12, 10.0, theta, z0=500.0)
    nrm = oracle.normals(dem, 10.0, "f64")
    # the plane falls along +row: n = (0, sin, cos) of the slope angle
    assert np.allclose(nrm[..., 0], 0.0, atol=1e-12)
    assert np.allclose(nrm[..., 1], math.sin(math.radians(theta)), atol=2e-6)
    assert np.allclose(nrm[..., 2], math.cos(math.radians(theta)), atol=2e-6)
    assert np.allclose(nrm[..., 3], theta, atol=2e-4)


def test_cone_slope_closed_form():
    dem = synth.cone_dem(41, 10.0, 38.0, z0=4000.0)
    nrm = oracle.normals(dem, 10.0, "f64")
    # away from the apex and the edges the central difference of a cone is the cone slope up to
    # curvature error O(1/r)
    r = np.hypot(*np.meshgrid(np.arange(41) - 20, np.arange(41) - 20, indexing="ij"))
    band = (r > 8) & (r < 18)
    assert np.max(np.abs(nrm[..., 3][band] - 38.0)) < 0.6
    # and the horizontal part of the normal points away from the apex
    rr, cc = np.meshgrid(np.arange(41) - 20, np.arange(41) - 20, indexing="ij")
    dot = nrm[..., 0] * cc + nrm[..., 1] * rr
    assert np.all(dot[band] > 0)


def test_release_mask_plane_and_bounds():
    for theta, expect in ((35.0, 1), (25.0, 0), (50.0, 0)):
        dem = synth.plane_dem(10, 10, 10.0, theta, z0=1000.0)
        nrm = oracle.normals(dem, 10.0)
        m = oracle.release_mask(nrm, dem, 30.0, 45.0, -np.inf, np.inf)
        assert np.all(m == expect), theta
    # elevation window is inclusive on both ends
    dem = synth.plane_dem(10, 4, 10.0, 35.0, z0=100.0)
    nrm = oracle.normals(dem, 10.0)
    zlo, zhi = float(dem[6, 0]), float(dem[2, 0])
    m = oracle.release_mask(nrm, dem, 30.0, 45.0, zlo, zhi)
    assert np.array_equal(m.any(axis=1), np.array([0, 0, 1, 1, 1, 1, 1, 0, 0, 0], bool))


def test_release_mask_bounds_are_inclusive():
    # flat ground has nz = 1 = cos(0): a range starting at 0 degrees keeps it
    flat = np.zeros((6, 5), np.float32)
    nrm = oracle.normals(flat, 10.0)
    assert np.all(oracle.release_mask(nrm, flat, 0.0, 10.0, -np.inf, np.inf) == 1)
    assert np.all(oracle.release_mask(nrm, flat, 0.5, 10.0, -np.inf, np.inf) == 0)
    # a range whose rounded cosine bound equals a cell's nz keeps that cell, at either end
    dem = synth.alpine_dem(64, 400.0, seed=21)
    nrm = oracle.normals(dem, 10.0)
    nz = nrm[..., 2]
    v = nz[10, 10]
    deg = math.degrees(math.acos(float(v)))
    assert np.float32(math.cos(np.float32(deg) * (math.pi / 180.0))) == v
    lo = oracle.release_mask(nrm, dem, float(np.float32(deg)), 89.0, -np.inf, np.inf)
    hi = oracle.release_mask(nrm, dem, 0.0, float(np.float32(deg)), -np.inf, np.inf)
    assert lo[10, 10] == 1 and hi[10, 10] == 1
    assert np.array_equal(lo.astype(bool) & hi.astype(bool), nz == v)


def test_release_mask_matches_slope_rule():
    w = synth.make_workload("tiny")
    nrm64 = oracle.normals(w.dem, w.cell_size, "f64")
    nrm = oracle.normals(w.dem, w.cell_size)
    m = oracle.release_mask(nrm, w.dem, 30.0, 45.0, w.z_min, w.z_max)
    slope = nrm64[..., 3]
    z = w.dem
    rule = (slope >= 30.0) & (slope <= 45.0) & (z >= w.z_min)
    # the cosine test and the angle test agree except within float rounding of the bounds
    near = (np.abs(slope - 30.0) < 1e-3) | (np.abs(slope - 45.0) < 1e-3)
    assert np.array_equal(m.astype(bool)[~near], rule[~near])
    assert 15000 < m.sum() < 25000


@pytest.mark.parametrize("shape,p", [((1, 1), 1.0), ((3, 7), 0.5), ((64, 65), 0.1), ((256, 256), 0.0),
                                     ((100, 3), 1.0)])
def test_compaction_matches_flatnonzero(shape, p):
    rng = np.random.default_rng(int(shape[0] * 1000 + shape[1]))
    m = (rng.random(shape) < p).astype(np.uint8)
    assert np.array_equal(oracle.compact(m), np.flatnonzero(m).astype(np.int32))
