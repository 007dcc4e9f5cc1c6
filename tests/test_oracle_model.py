"""Pins of the oracle's trajectory model (section 5.2, the trajectory node) against closed forms,
independent library routines and brute force.

* friction law: on an exact plane with no drag, v^2 after n steps is 2 g n dl (tan(theta) - mu), i.e.
  2 g s (sin(theta) - mu cos(theta)) over path length s; with Voellmy drag the speed converges to the
  terminal speed sqrt(xi h (sin(theta) - mu cos(theta))); on a plane running out onto flat ground the
  Coulomb energy line stops the particle after a horizontal distance H/mu; the kinetic height never
  exceeds the release energy line z_r - mu * (horizontal path);
* runout-angle stop: on the flat the particle stops where the line to the release point falls below
  the runout angle;
* the path: heights and gradients equal scipy's bilinear interpolant of the texel centres; each new
  direction is the normalised blend persistence * previous + (1 - persistence) * downslope + randomness
  * (uniforms from rocRAND's Philox4x32-10); each move is one step along it;
* accumulation: hit counts, per-cell max speed and step statistics equal a brute-force rebuild from
  per-particle traces on 8x8 grids; runs superpose over disjoint release masks; zero steps leave
  the particles in their release cells; a cone gives a D4-symmetric runout.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from tests.support.philox_ref import philox_blocks

INF = float("inf")
G32 = float(np.float32(9.81))


def g_of(prec):
    return G32 if prec == "f32" else 9.81


def f32(v):
    """Parameters cross into the model as binary32; closed forms use the same rounded values."""
    return float(np.float32(v))


def exact_plane(h, w, k=7.0, z0=None):
    """Plane falling by exactly k metres per row, all texel heights exact in float32."""
    z0 = k * h if z0 is None else z0
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(z0 - k * r, (h, w)).astype(np.float32)


def exact_plane_to_flat(h, w, kink, k=7.0):
    r = np.arange(h, dtype=np.float64)[:, None]
    return np.broadcast_to(np.maximum(k * (kink - r), 0.0), (h, w)).astype(np.float32)


# ------------------------------------------------------------------------------------------ friction law

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mu", [0.0, 0.2, 0.55])
def test_plane_coulomb_closed_form(prec, mu):
    cs, k = 10.0, 7.0
    tan = k / cs
    dem = exact_plane(400, 9, k)
    p = oracle.make_params(mu=mu, xi=INF, flow_height=1.0, persistence=0.9, randomness=0.0)
    tr = oracle.trace(dem, cs, p, r=2, c=4, replica=0, step_limit=300, seed=7, prec=prec)
    assert tr.reason == oracle.END_LIMIT and len(tr.rows) == 301
    assert np.all(tr.x == 4.5)                     # straight down the fall line
    assert np.allclose(np.diff(tr.y), 1.0, atol=1e-5)
    n = np.arange(301)
    theta = math.atan(tan)
    s = n * cs / math.cos(theta)                   # path length
    closed = 2 * g_of(prec) * s * (math.sin(theta) - f32(mu) * math.cos(theta))
    rtol = 3e-5 if prec == "f32" else 1e-12
    assert np.allclose(tr.v2, closed, rtol=rtol, atol=1e-3 if prec == "f32" else 1e-9)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mu,xi,h", [(0.25, 1500.0, 1.0), (0.1, 500.0, 2.5), (0.4, 3000.0, 0.5)])
def test_voellmy_terminal_speed(prec, mu, xi, h):
    cs, k = 10.0, 7.0
    dem = exact_plane(260, 5, k)
    p = oracle.make_params(mu=mu, xi=xi, flow_height=h, persistence=0.9, randomness=0.0)
    tr = oracle.trace(dem, cs, p, r=1, c=2, replica=0, step_limit=250, seed=1, prec=prec)
    theta = math.atan(k / cs)
    vstar2 = f32(xi) * f32(h) * (math.sin(theta) - f32(mu) * math.cos(theta))
    rtol = 2e-5 if prec == "f32" else 1e-9
    assert abs(tr.v2[-1] / vstar2 - 1) < rtol
    # monotone approach from below
    assert np.all(np.diff(tr.v2) >= -1e-9 * vstar2)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mu", [0.15, 0.25, 0.5])
def test_plane_to_flat_stop_distance(prec, mu):
    cs, k, kink, r0 = 10.0, 7.0, 40, 2
    dem = exact_plane_to_flat(40 + 300, 5, kink, k)
    p = oracle.make_params(mu=mu, xi=INF, flow_height=1.0, persistence=0.9, randomness=0.0)
    tr = oracle.trace(dem, cs, p, r=r0, c=2, replica=0, step_limit=1000, seed=1, prec=prec)
    assert tr.reason == oracle.END_STOP
    zr = k * (kink - r0)
    # energy line: the particle stops after a horizontal distance of z_r / mu (one step of rounding)
    n_expect = math.ceil(zr / (f32(mu) * cs)) - 1
    assert abs((len(tr.rows) - 1) - n_expect) <= 1
    assert tr.steps == len(tr.rows)                 # the rejected step was entered


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_runout_angle_stop(prec):
    cs, k, kink, r0 = 10.0, 7.0, 40, 2
    dem = exact_plane_to_flat(40 + 200, 5, kink, k)
    tan_alpha = 0.5
    p = oracle.make_params(mu=0.0, xi=INF, flow_height=1.0, persistence=0.9, randomness=0.0,
                           tan_alpha=tan_alpha)
    tr = oracle.trace(dem, cs, p, r=r0, c=2, replica=0, step_limit=1000, seed=1, prec=prec)
    assert tr.reason == oracle.END_STOP
    zr = k * (kink - r0)
    # on the flat, the angle to the release point falls below alpha at distance z_r / (tan(alpha) cs)
    assert abs((len(tr.rows) - 1) - math.floor(zr / (tan_alpha * cs))) <= 1
    # without the runout-angle stop, the frictionless particle runs to the grid edge
    p2 = oracle.make_params(mu=0.0, xi=INF, flow_height=1.0, persistence=0.9, randomness=0.0)
    assert oracle.trace(dem, cs, p2, r=r0, c=2, replica=0, step_limit=1000, seed=1, prec=prec).reason \
        == oracle.END_EXIT


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("xi", [INF, 1200.0])
def test_energy_line(prec, xi):
    cs, mu = 10.0, 0.12
    dem = synth.alpine_dem(128, 900.0, seed=11)
    p = oracle.make_params(mu=mu, xi=xi, flow_height=1.5, persistence=0.8, randomness=0.25)
    rng = np.random.default_rng(3)
    g = g_of(prec)
    long_paths = 0
    for _ in range(40):
        r, c = rng.integers(10, 118, size=2)
        tr = oracle.trace(dem, cs, p, r=int(r), c=int(c), replica=int(rng.integers(0, 99)), step_limit=400,
                          seed=5, prec=prec)
        n = np.arange(len(tr.rows))
        e = (tr.z[0] - tr.z) - f32(mu) * n * cs   # release energy line minus terrain, metres
        kin = tr.v2 / (2 * g)
        tol = (2e-3 + 1e-5 * np.abs(e)) if prec == "f32" else 1e-9 * (1 + np.abs(e))
        if xi == INF:
            assert np.all(np.abs(kin - e) <= tol)
        else:
            assert np.all(kin <= e + tol)
            if len(n) > 3:
                assert np.all(kin[2:] < e[2:])     # drag takes energy strictly
        long_paths += len(n) > (20 if xi == INF else 8)
    assert long_paths > 10


# ------------------------------------------------------------------------------------------ the path

def _philox_uniforms(steps, replica, cell, run, seed):
    """The model's two uniforms in [-1, 1) for each step, from rocRAND's Philox4x32-10."""
    rows = np.array([[n >> 1, replica, cell, run, seed & 0xFFFFFFFF, seed >> 32] for n in range(steps)],
                    np.uint32).reshape(-1, 6)
    o = philox_blocks(rows).astype(np.int64) if steps else np.zeros((0, 4), np.int64)
    odd = (np.arange(steps) & 1).astype(bool)
    ux = np.where(odd, o[:, 2], o[:, 0])
    uy = np.where(odd, o[:, 3], o[:, 1])
    return 2.0 * (ux >> 8) * 2.0 ** -24 - 1.0, 2.0 * (uy >> 8) * 2.0 ** -24 - 1.0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_path_bilinear_and_direction_blend(prec):
    cs = 10.0
    dem = synth.alpine_dem(96, 500.0, seed=12)
    h, w = dem.shape
    per, rnd, L = 0.7, 0.3, 0.8
    p = oracle.make_params(mu=0.05, xi=INF, flow_height=1.0, persistence=per, randomness=rnd, step_cells=L)
    f = RegularGridInterpolator((np.arange(h) + 0.5, np.arange(w) + 0.5), dem.astype(np.float64))
    seed, run = 0x0123456789ABCDEF, 4
    zt, gt, dt, mt = (1e-9, 1e-6, 1e-7, 1e-9) if prec == "f64" else (2e-4, 5e-3, 2e-5, 2e-5)
    checked = paths = 0
    rng = np.random.default_rng(12)
    for _ in range(12):
        r, c, j = (int(v) for v in rng.integers(5, 90, size=3))
        tr = oracle.trace(dem, cs, p, r=r, c=c, replica=j, step_limit=120, seed=seed, run=run, prec=prec)
        rows = tr.rows.astype(np.float64)
        paths += len(rows) > 10
        rxs, rys = _philox_uniforms(len(rows), j, r * w + c, run, seed)
        for i in range(len(rows)):
            x, y, z, gx, gy = rows[i, :5]
            inside = 0.5 < x < w - 0.5 and 0.5 < y < h - 0.5
            if inside:
                assert abs(z - f((y, x))) < zt * max(1.0, abs(z))
                fx, fy = (x - 0.5) % 1.0, (y - 0.5) % 1.0
                if 1e-3 < fx < 1 - 1e-3 and 1e-3 < fy < 1 - 1e-3:
                    e = 1e-5
                    gxf = (f((y, x + e)) - f((y, x - e))) / (2 * e)
                    gyf = (f((y + e, x)) - f((y - e, x))) / (2 * e)
                    assert abs(gx - gxf) < gt * max(1.0, abs(gxf))
                    assert abs(gy - gyf) < gt * max(1.0, abs(gyf))
                    checked += 1
            if i + 1 < len(rows):
                rx, ry = rxs[i], rys[i]
                gn = math.hypot(gx, gy)
                ex, ey = (-gx / gn, -gy / gn) if gn > 0 else (0.0, 0.0)
                pf, rf = f32(per), f32(rnd)
                wx = pf * rows[i, 5] + (1 - pf) * ex + rf * rx
                wy = pf * rows[i, 6] + (1 - pf) * ey + rf * ry
                wn = math.hypot(wx, wy)
                assert abs(rows[i + 1, 5] - wx / wn) < dt and abs(rows[i + 1, 6] - wy / wn) < dt
                assert abs(rows[i + 1, 0] - (x + f32(L) * rows[i + 1, 5])) < mt * max(1.0, x)
                assert abs(rows[i + 1, 1] - (y + f32(L) * rows[i + 1, 6])) < mt * max(1.0, y)
    assert paths >= 4 and checked > 100


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_border_strip_is_clamped(prec):
    # Within half a cell of the grid edge the height patch is extended flat from the edge texels,
    # the same as interpolating at the query point clamped into the texel-centre grid.
    cs, h, w = 10.0, 12, 9
    rr, cc = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    cases = (((3.0 * cc + 0.01 * rr).astype(np.float32), ((5, 2), (8, 3)), "x"),        # falls to -x
             ((3.0 * (h - 1 - rr) + 0.01 * cc).astype(np.float32), ((h - 3, 4), (h - 4, 2)), "y"))
    p = oracle.make_params(mu=0.0, xi=INF, persistence=0.9, randomness=0.0, step_cells=0.7)
    for dem, starts, axis in cases:
        f = RegularGridInterpolator((np.arange(h) + 0.5, np.arange(w) + 0.5), dem.astype(np.float64))
        strip_rows = 0
        for r, c in starts:
            tr = oracle.trace(dem, cs, p, r=r, c=c, replica=0, step_limit=50, seed=1, prec=prec)
            assert tr.reason == oracle.END_EXIT
            for x, y, z, gx, gy in tr.rows[:, :5].astype(np.float64):
                q = (min(max(y, 0.5), h - 0.5), min(max(x, 0.5), w - 0.5))
                assert abs(z - f(q)) < (1e-4 if prec == "f32" else 1e-10)
                if axis == "x" and x < 0.5:
                    assert gx == 0.0
                    strip_rows += 1
                if axis == "y" and y > h - 0.5:
                    assert gy == 0.0
                    strip_rows += 1
        assert strip_rows >= 2


def test_initial_direction_is_downslope_and_flat_is_still():
    cs = 10.0
    dem = exact_plane(20, 20, 7.0)
    p = oracle.make_params(persistence=1.0, randomness=0.0, mu=0.0, xi=INF)
    tr = oracle.trace(dem, cs, p, r=3, c=9, replica=0, step_limit=5, seed=1)
    assert tr.rows[0, 5] == 0.0 and abs(tr.rows[0, 6] - 1.0) < 1e-6
    # flat ground, no randomness: no direction, the particle does not move, mu = 0 -> runs to the limit
    flat = np.zeros((8, 8), np.float32)
    tr = oracle.trace(flat, cs, oracle.make_params(mu=0.0, randomness=0.0, xi=INF), r=3, c=3, replica=0,
                      step_limit=10, seed=1)
    assert tr.reason == oracle.END_STOP or (tr.reason == oracle.END_LIMIT and np.all(tr.x == 3.5))


# ------------------------------------------------------------------------------------------ accumulation

def _rebuild(dem, mask, cs, p, P, S, seed, run, prec):
    h, w = dem.shape
    counts = np.zeros((h, w), np.int64)
    vmax2 = np.zeros((h, w), np.float64 if prec == "f64" else np.float32)
    steps = 0
    ends = [0, 0, 0]
    for cell in np.flatnonzero(mask):
        r, c = divmod(int(cell), w)
        for j in range(P):
            tr = oracle.trace(dem, cs, p, r, c, j, S, seed, run, prec)
            steps += tr.steps
            ends[tr.reason] += 1
            cells = np.floor(tr.y).astype(int) * w + np.floor(tr.x).astype(int)
            entered = np.ones(len(cells), bool)
            entered[1:] = cells[1:] != cells[:-1]
            np.add.at(counts.ravel(), cells[entered], 1)
            np.maximum.at(vmax2.ravel(), cells, tr.v2.astype(vmax2.dtype))
    return counts, np.sqrt(vmax2), steps, ends


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_bruteforce_8x8(prec):
    rng = np.random.default_rng(8)
    for case in range(10):
        base = exact_plane(8, 8, float(rng.uniform(2, 9)))
        if case % 2:
            base = base.T.copy()
        dem = (base + rng.standard_normal((8, 8)) * rng.uniform(0, 6)).astype(np.float32)
        mask = (rng.random((8, 8)) < 0.35).astype(np.uint8)
        xi = [INF, 500.0, 3000.0][case % 3]
        p = oracle.make_params(mu=float(rng.uniform(0, 0.5)), xi=xi, flow_height=float(rng.uniform(0.5, 3)),
                               persistence=float(rng.uniform(0, 1)), randomness=float(rng.uniform(0, 0.6)),
                               step_cells=float([1.0, 0.5, 0.75][case % 3]),
                               tan_alpha=[-1.0, 0.3][case % 2])
        P, S, seed, run = 3, 40, int(rng.integers(0, 2**63)), case
        res = oracle.trajectories(dem, mask, 5.0, p, P, S, seed, run, prec)
        counts, vmax, steps, ends = _rebuild(dem, mask, 5.0, p, P, S, seed, run, prec)
        assert np.array_equal(res.counts, counts)
        assert np.array_equal(res.vmax, vmax.astype(res.vmax.dtype))
        assert res.steps == steps
        assert [res.n_limit, res.n_exit, res.n_stop] == ends
        assert res.n_exit + res.n_stop + res.n_limit == P * int(mask.sum())


def test_superposition_over_masks():
    w = synth.make_workload("tiny")
    nrm = oracle.normals(w.dem, w.cell_size)
    m = oracle.release_mask(nrm, w.dem, 30, 45, w.z_min, w.z_max)
    rng = np.random.default_rng(1)
    keep = (rng.random(m.shape) < 0.02) & (m == 1)
    a = (keep & (rng.random(m.shape) < 0.5)).astype(np.uint8)
    b = (keep & (a == 0)).astype(np.uint8)
    p = oracle.make_params(**w.params)
    ra = oracle.trajectories(w.dem, a, w.cell_size, p, 4, 500, 9)
    rb = oracle.trajectories(w.dem, b, w.cell_size, p, 4, 500, 9)
    rab = oracle.trajectories(w.dem, (a | b).astype(np.uint8), w.cell_size, p, 4, 500, 9)
    assert np.array_equal(rab.counts, ra.counts + rb.counts)
    assert np.array_equal(rab.vmax, np.maximum(ra.vmax, rb.vmax))
    assert rab.steps == ra.steps + rb.steps


def test_zero_steps_and_empty_mask():
    dem = synth.alpine_dem(32, 300.0, seed=3)
    mask = np.zeros((32, 32), np.uint8)
    mask[5, 7] = mask[20, 3] = 1
    p = oracle.make_params()
    res = oracle.trajectories(dem, mask, 10.0, p, 5, 0, 1)
    assert np.array_equal(res.counts, 5 * mask.astype(np.uint32))
    assert np.all(res.vmax == 0) and res.steps == 0 and res.n_limit == 10
    res = oracle.trajectories(dem, np.zeros_like(mask), 10.0, p, 5, 100, 1)
    assert res.counts.sum() == 0 and res.steps == 0


def test_cone_runout_is_d4_symmetric():
    n, h = 161, 80
    dem = synth.cone_dem(n, 10.0, 38.0, z0=400.0)
    rr, cc = np.meshgrid(np.arange(n) - h, np.arange(n) - h, indexing="ij")
    ring = (np.hypot(rr, cc) >= 4) & (np.hypot(rr, cc) < 6)
    p = oracle.make_params(mu=0.6, xi=INF, persistence=0.9, randomness=0.0)
    res = oracle.trajectories(dem, ring.astype(np.uint8), 10.0, p, 1, 500, 1)
    assert res.n_exit == 0 and res.n_limit == 0
    assert np.hypot(rr, cc)[res.counts > 0].max() > 55          # ran down the cone onto the flat

    def stop_radius(a, b):
        tr = oracle.trace(dem, 10.0, p, h + a, h + b, 0, 500, 1)
        return math.hypot(tr.x[-1] - (h + 0.5), tr.y[-1] - (h + 0.5))

    # every ray and its images under the rotations and reflections of the square stop at the same radius
    for a, b in zip(*np.nonzero(ring)):
        a, b = int(a) - h, int(b) - h
        base = stop_radius(a, b)
        for a2, b2 in ((-b, a), (-a, -b), (b, -a), (b, a), (a, -b), (-a, b)):
            assert abs(stop_radius(a2, b2) - base) <= 1.0
