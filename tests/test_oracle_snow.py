"""Pins of the oracle's snow-cover node (section 5.1: snow line, maximal steepness and blend factors of
the transition zones decide a per-texel snow alpha from the terrain alone).

* without blend zones the alpha is the indicator {slope <= max_slope and z >= snow_line}, which is the
  release map over the slope window [0, max_slope] and elevations [snow_line, +inf);
* the elevation ramp on flat ground with heights on a line equals the exact fraction (z - line) / blend;
* the steepness ramp is linear in nz between cos(max_slope) and cos(max_slope - slope_blend): hand-set
  nz values at k/8 of the way give k/8;
* on alpine terrain the alpha is 0 below the snow line and on slopes steeper than the maximum (slope
  from the normals' angle channel, an independent atan route), 1 above the blend zones, and never
  decreases with height when the slope is held.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def n4(nz):
    out = np.zeros(nz.shape + (4,), np.float64)
    out[..., 2] = nz
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_no_blend_is_the_release_map_indicator(prec):
    dem = synth.alpine_dem(96, 1500.0, seed=14)
    nrm = oracle.normals(dem, 10.0, prec=prec)
    line = float(np.quantile(dem, 0.45))
    for smax in (25.0, 38.5, 60.0):
        a = oracle.snow_cover(nrm, dem, line, 0.0, smax, 0.0, prec=prec)
        m = oracle.release_mask(nrm, dem, 0.0, smax, line, float("inf"), prec=prec)
        assert 0 < m.sum() < m.size
        np.testing.assert_array_equal(a, m.astype(a.dtype))


def test_elevation_ramp_on_a_line():
    h, w = 3, 40
    z = 1000.0 + 12.5 * np.arange(w)          # dyadic heights
    dem = np.broadcast_to(z, (h, w)).astype(np.float32)
    line, blend = 1100.0, 200.0
    a = oracle.snow_cover(n4(np.ones((h, w))), dem, line, blend, 45.0, 10.0, prec="f64")
    for c in range(w):
        t = (Fraction(z[c]) - Fraction(line)) / Fraction(blend)
        want = float(min(max(t, Fraction(0)), Fraction(1)))
        assert np.all(np.abs(a[:, c] - want) <= 1e-15)


@pytest.mark.parametrize("smax,blend", [(40.0, 10.0), (35.0, 0.5), (80.0, 30.0)])
def test_steepness_ramp_is_linear_in_nz(smax, blend):
    lo, hi = math.cos(math.radians(smax)), math.cos(math.radians(smax - blend))
    ks = np.arange(-3, 12)
    nz = lo + (ks / 8.0) * (hi - lo)
    dem = np.full((1, len(ks)), 5000.0, np.float32)
    a = oracle.snow_cover(n4(nz[None, :]), dem, 0.0, 0.0, smax, blend, prec="f64")[0]
    want = np.clip(ks / 8.0, 0.0, 1.0)
    np.testing.assert_allclose(a, want, rtol=0, atol=1e-9)


def test_alpine_limits_and_monotone_in_height():
    dem = synth.alpine_dem(128, 2000.0, seed=3)
    nrm = oracle.normals(dem, 10.0, prec="f64")
    slope = nrm[..., 3]
    line, zb, smax, sb = float(np.quantile(dem, 0.3)), 150.0, 45.0, 12.0
    a = oracle.snow_cover(nrm, dem, line, zb, smax, sb, prec="f64")
    assert np.all((a >= 0) & (a <= 1))
    assert np.all(a[dem <= line] == 0)
    assert np.all(a[slope > smax + 1e-6] == 0)
    full = (dem >= line + zb) & (slope < smax - sb - 1e-6)
    assert full.sum() > 100 and np.all(a[full] == 1)
    mid = (a > 0) & (a < 1)
    assert mid.sum() > 100
    # raising every height keeps the slopes and never lowers the alpha
    b = oracle.snow_cover(nrm, dem + np.float32(40.0), line, zb, smax, sb, prec="f64")
    assert np.all(b >= a)
