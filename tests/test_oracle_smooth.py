"""Pins of the oracle's smooth variant (deposit of the released mass at each particle's resting point) and
of its gradient with respect to mu, xi, h and the per-cell release mass.

* resting point: on a plane running out onto flat ground (no drag, no randomness) the Coulomb energy line
  reaches zero at horizontal distance z_r / mu from the release point, and the bilinear splat keeps the
  first moment, so the deposit's centroid is that closed form (not only to one step: the fractional last
  step makes the resting point continuous);
* conservation: the deposit holds exactly the mass of the particles that did not leave the grid (and the
  fixed-point raster agrees with the unquantised one to 2^-24 per splat corner);
* velocity splat: its total equals the sum of speeds over per-particle traces, and its first moments put each
  speed at the position its step moved to;
* gradient: the closed-form derivative -z_r / (mu^2 cs) of the resting point on the plane-to-flat; the
  reverse sweep against an independent forward-mode derivation; against central finite differences of
  the binary64 forward; the mass gradient against the exact linear response.
"""
import math

import numpy as np
import pytest

import oracle
import synth

INF = float("inf")


def f32(v):
    return float(np.float32(v))


def plane_to_flat(h, w, kink, k=7.0):
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(np.maximum(k * (kink - r), 0.0), (h, w)).astype(np.float32)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mu", [0.15, 0.22, 0.37])
def test_resting_point_closed_form(prec, mu):
    cs, k, kink = 10.0, 7.0, 40
    dem = plane_to_flat(400, 9, kink, k)
    mask = np.zeros_like(dem, np.uint8)
    mask[3, 4] = 1
    p = oracle.make_params(mu=mu, xi=INF, persistence=0.9, randomness=0.0)
    res = oracle.smooth_forward(dem, mask, cs, p, 3, 2000, 1, prec=prec)
    assert res.n_stop == 3
    zr = k * (kink - 3)
    y_star = 3.5 + zr / (f32(mu) * cs)                 # cell units along +row
    rows = np.arange(dem.shape[0]) + 0.5
    cols = np.arange(dem.shape[1]) + 0.5
    tot = res.dep.sum()
    assert abs(tot - 1.0) < 1e-6
    yc = (res.dep.sum(axis=1) * rows).sum() / tot
    xc = (res.dep.sum(axis=0) * cols).sum() / tot
    tol = 2e-4 if prec == "f32" else 1e-9
    assert abs(yc - y_star) < tol * y_star
    assert abs(xc - 4.5) < 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_mass_conservation_and_fixed_point(prec):
    w = synth.make_workload("tiny")
    mask = oracle.release_mask(oracle.normals(w.dem, 10.0), w.dem, 30, 45, w.z_min, w.z_max)
    sub = np.zeros_like(mask)
    sub.ravel()[np.flatnonzero(mask)[::40]] = 1
    mass = np.random.default_rng(2).uniform(0.5, 2.0, mask.shape).astype(np.float32)
    P = 6
    res = oracle.smooth_forward(w.dem, sub, 10.0, oracle.make_params(**w.params), P, 2000, 4, mass=mass, prec=prec)
    # mass that stayed on the grid: rebuild which particles exited from the plain run of each cell
    released = 0.0
    for cell in np.flatnonzero(sub):
        one = np.zeros_like(sub)
        one.ravel()[cell] = 1
        r1 = oracle.trajectories(w.dem, one, 10.0, oracle.make_params(**w.params), P, 2000, 4)
        released += (P - r1.n_exit) * float(np.float32(mass.ravel()[cell]) / np.float32(P))
    assert res.n_exit > 0
    assert abs(res.dep.sum() - released) < 1e-4 * released
    n_part = int(sub.sum()) * P
    assert abs(res.dep_q.sum() * 2.0 ** -24 - res.dep.sum()) < 4 * n_part * 2.0 ** -24 + 1e-6 * released


def test_velocity_splat_matches_traces():
    dem = synth.alpine_dem(64, 500.0, seed=5)
    mask = np.zeros((64, 64), np.uint8)
    mask[10:14, 20:24] = 1
    p = oracle.make_params(mu=0.1, xi=1500.0, randomness=0.2)
    P = 3
    res = oracle.smooth_forward(dem, mask, 10.0, p, P, 300, 9, vel_splat=True, prec="f64")
    tot = 0.0
    for cell in np.flatnonzero(mask):
        r, c = divmod(int(cell), 64)
        for j in range(P):
            tr = oracle.trace(dem, 10.0, p, r, c, j, 300, 9, prec="f64")
            tot += (1.0 / P) * np.sqrt(tr.v2[1:]).sum()
    assert abs(res.vel.sum() - tot) < 1e-9 * tot
    assert tot > 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_velocity_splat_first_moments_put_it_after_the_move(prec):
    """Where each speed lands. A bilinear splat reproduces linear functions: for a point p at least half a
    texel inside the grid, the weights w_q(p) of its four texels satisfy sum_q w_q (c_q + 1/2) = p_x and
    sum_q w_q (r_q + 1/2) = p_y. So the raster's first moments are sum mp v_k x_k and sum mp v_k y_k over the
    accepted steps k, with (x_k, y_k) the position the step moved to and v_k the speed after it. A splat at
    the position before the move, or at the release point, gives other moments (checked to differ here by
    far more than the tolerance), which the total alone cannot show."""
    n = 160
    dem = synth.alpine_dem(n, 900.0, seed=5)
    mask = np.zeros((n, n), np.uint8)
    mask[78:82, 78:82] = 1
    p = oracle.make_params(mu=0.1, xi=1500.0, randomness=0.2)
    P, S = 3, 60  # paths of at most 60 one-cell steps stay inside [18, 142]^2
    res = oracle.smooth_forward(dem, mask, 10.0, p, P, S, 9, vel_splat=True, prec=prec)
    mp = 1.0 / P
    m0 = mx = my = 0.0
    pre_x = pre_y = rel_x = 0.0
    for cell in np.flatnonzero(mask):
        r, c = divmod(int(cell), n)
        for j in range(P):
            tr = oracle.trace(dem, 10.0, p, r, c, j, S, 9, prec=prec)
            x, y = tr.x.astype(np.float64), tr.y.astype(np.float64)
            v = np.sqrt(tr.v2[1:].astype(np.float64))
            assert x.min() > 0.5 and x.max() < n - 0.5 and y.min() > 0.5 and y.max() < n - 0.5
            m0 += mp * v.sum()
            mx += mp * (v * x[1:]).sum()
            my += mp * (v * y[1:]).sum()
            pre_x += mp * (v * x[:-1]).sum()
            pre_y += mp * (v * y[:-1]).sum()
            rel_x += mp * (v * x[0]).sum()
    centres = np.arange(n) + 0.5
    vel = res.vel.astype(np.float64)
    tol = 1e-9 if prec == "f64" else 2e-6
    assert abs(vel.sum() - m0) <= tol * m0
    assert abs((vel.sum(axis=0) * centres).sum() - mx) <= tol * mx
    assert abs((vel.sum(axis=1) * centres).sum() - my) <= tol * my
    # the moments tell the placements apart
    assert abs(pre_x - mx) + abs(pre_y - my) > 1e3 * tol * (mx + my)
    assert abs(rel_x - mx) > 1e3 * tol * mx
    # the fixed-point raster carries the same splat: within 2^-24 per corner of every splat
    n_splat = int(res.steps)
    assert abs(res.vel_q.sum() * 2.0 ** -24 - vel.sum()) <= 4 * n_splat * 2.0 ** -24 + tol * m0


@pytest.mark.parametrize("mu", [0.15, 0.3])
def test_gradient_closed_form_first_moment(mu):
    """L = sum over texels of (row + 1/2) * D is the sum of mp * y* (first moment), so dL/dmu is
    sum mp * dy*/dmu = -N mp z_r / (mu^2 cs) on the plane-to-flat."""
    cs, k, kink = 10.0, 7.0, 40
    dem = plane_to_flat(400, 9, kink, k)
    mask = np.zeros_like(dem, np.uint8)
    mask[3, 4] = 1
    p = oracle.make_params(mu=mu, xi=INF, persistence=0.9, randomness=0.0)
    gD = np.broadcast_to((np.arange(400) + 0.5)[:, None], dem.shape).astype(np.float32)
    zr = k * (kink - 3)
    expect = -zr / (f32(mu) ** 2 * cs)                  # N mp = 2 particles x mass 1/2 = 1
    for prec, tol in (("f64", 1e-9), ("f32", 1e-4)):
        g = oracle.smooth_backward(dem, mask, cs, p, 2, 2000, 1, gD, prec=prec)
        assert abs(g.dmu / expect - 1) < tol, prec
        assert g.dxi == 0.0
    t = oracle.smooth_tangent(dem, mask, cs, p, 2, 2000, 1, gD)
    assert abs(t[0] / expect - 1) < 1e-9


def _calib_case(seed=5, P=6):
    dem = synth.alpine_dem(96, 700.0, seed=seed)
    sl = synth.slope_deg(dem, 10.0)
    mask = ((sl >= 28) & (sl <= 45) & (dem >= np.quantile(dem, 0.6))).astype(np.uint8)
    rr, cc = np.meshgrid(np.arange(96), np.arange(96), indexing="ij")
    mask &= ((rr > 20) & (rr < 76) & (cc > 20) & (cc < 76)).astype(np.uint8)
    mass = np.random.default_rng(seed).uniform(0.5, 1.5, dem.shape).astype(np.float32)
    gD = np.random.default_rng(seed + 1).standard_normal(dem.shape).astype(np.float32)
    return dem, mask, mass, gD, P


def test_adjoint_equals_forward_mode():
    dem, mask, mass, gD, P = _calib_case()
    for xi in (1800.0, INF):
        p = oracle.make_params(mu=0.22, xi=xi, flow_height=1.3, randomness=0.16)
        g = oracle.smooth_backward(dem, mask, 10.0, p, P, 1500, 3, gD, mass=mass, prec="f64")
        t = oracle.smooth_tangent(dem, mask, 10.0, p, P, 1500, 3, gD, mass=mass)
        assert abs(g.dmu - t[0]) <= 1e-10 * abs(t[0])
        assert abs(g.dxi - t[1]) <= 1e-10 * abs(t[1]) + 1e-300
        assert abs(g.dh - t[2]) <= 1e-10 * abs(t[2]) + 1e-300
        if xi == INF:
            assert g.dxi == 0.0 and g.dh == 0.0


def _loss(dem, mask, mass, gD, P, **kw):
    p = oracle.make_params(**kw)
    res = oracle.smooth_forward(dem, mask, 10.0, p, P, 1500, 3, mass=mass, prec="f64")
    return float((gD.astype(np.float64) * res.dep).sum())


@pytest.mark.parametrize("name", ["mu", "xi", "flow_height"])
def test_adjoint_matches_central_differences(name):
    """Central differences of the binary64 forward with steps of a few binary32 ulps (parameters are
    binary32 at the boundary), per particle, over the particles whose end (reason, steps completed) is
    the same on both sides: the loss is piecewise smooth (a particle that barely reaches a crest may
    restart downhill), and the adjoint is the derivative of the smooth pieces."""
    dem, mask, mass, gD, P = _calib_case()
    base = dict(mu=0.22, xi=1800.0, flow_height=1.3, randomness=0.16)
    g = oracle.smooth_backward(dem, mask, 10.0, oracle.make_params(**base), P, 1500, 3, gD, mass=mass, prec="f64")
    col = {"mu": 0, "xi": 1, "flow_height": 2}[name]
    for ulps in (4, 16):
        v = np.float32(base[name])
        hi, lo = v, v
        for _ in range(ulps):
            hi = np.nextafter(hi, np.float32(np.inf))
            lo = np.nextafter(lo, np.float32(-np.inf))
        Lh, rh, sh = oracle.smooth_particles(dem, mask, 10.0, oracle.make_params(**dict(base, **{name: float(hi)})), P,
                                             1500, 3, gD, mass=mass)
        Ll, rl, sl = oracle.smooth_particles(dem, mask, 10.0, oracle.make_params(**dict(base, **{name: float(lo)})), P,
                                             1500, 3, gD, mass=mass)
        same = (rh == rl) & (sh == sl)
        assert same.mean() > 0.99
        fd = (Lh - Ll) / (float(hi) - float(lo))
        adj = g.per_particle[:, col]
        assert abs(fd[same].sum() - adj[same].sum()) <= 1e-3 * abs(adj[same].sum()), (name, ulps)
        # particle by particle, too
        big = same & (np.abs(adj) > 1e-6 * np.abs(adj).max())
        assert np.allclose(fd[big], adj[big], rtol=1e-3, atol=1e-6 * np.abs(adj).max())


def test_mass_gradient_is_exact_linear_response():
    dem, mask, mass, gD, P = _calib_case()
    p = dict(mu=0.22, xi=1800.0, flow_height=1.3, randomness=0.16)
    g = oracle.smooth_backward(dem, mask, 10.0, oracle.make_params(**p), P, 1500, 3, gD, mass=mass, prec="f64")
    base = _loss(dem, mask, mass, gD, P, **p)
    cells = np.flatnonzero(mask)[::37][:8]
    for cell in cells:
        m2 = mass.copy()
        m2.ravel()[cell] = np.float32(m2.ravel()[cell] * 2)   # exact doubling
        d = (_loss(dem, mask, m2, gD, P, **p) - base) / float(mass.ravel()[cell])
        assert abs(d - g.dmass.ravel()[cell]) <= 1e-9 * max(1.0, abs(d))
    assert np.all(g.dmass.ravel()[np.flatnonzero(mask == 0)] == 0)


def test_fp32_vs_fp64_gradient_stated():
    """The FP32 adjoint follows the FP64 one except on particles whose FP32 path diverges (a different
    texel edge crossing); stated as the diverged fraction and the error against the sum of |terms|."""
    dem, mask, mass, gD, P = _calib_case()
    p = oracle.make_params(mu=0.22, xi=1800.0, flow_height=1.3, randomness=0.16)
    g32 = oracle.smooth_backward(dem, mask, 10.0, p, P, 1500, 3, gD, mass=mass, prec="f32")
    g64 = oracle.smooth_backward(dem, mask, 10.0, p, P, 1500, 3, gD, mass=mass, prec="f64")
    a32, a64 = g32.per_particle.astype(np.float64), g64.per_particle
    diverged = np.abs(a32[:, 0] - a64[:, 0]) > 1e-3 * np.abs(a64[:, 0]) + 1e-9
    assert diverged.mean() < 0.03
    for col, name in ((0, "dmu"), (1, "dxi")):
        scale = np.abs(a64[:, col]).sum()
        assert abs(getattr(g32, name) - getattr(g64, name)) < 0.05 * scale
        # on the particles whose paths agree, the per-particle terms agree to FP32 rounding
        ok = ~diverged
        assert np.allclose(a32[ok, col], a64[ok, col], rtol=2e-3, atol=1e-6 * scale)
