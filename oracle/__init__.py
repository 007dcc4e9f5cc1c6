"""CPU oracle for the avalanche overlay hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this
package. The product package (``paper_2506_23364_amd``) never imports it and shares no code with it.

Two twins of one plain C source (``avl_oracle.c``): the FP32 oracle, which the GPU path must match
bit-exactly on integer outputs, and the FP64 twin, which states the FP32 error. Both are loaded through
ctypes from ``liboracle_f32.so`` / ``liboracle_f64.so`` next to this file (built by ``build.py``).

Parity status of each function is recorded in the design notes; every function here is pinned by a
test in ``tests/test_oracle_*.py`` against something other than itself (rocRAND's Philox, numpy's
gradient and flatnonzero, closed forms of the friction law, scipy's bilinear interpolant, invariants).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

END_LIMIT, END_EXIT, END_STOP = 0, 1, 2


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("mu", ctypes.c_float), ("xi", ctypes.c_float), ("flow_height", ctypes.c_float),
        ("persistence", ctypes.c_float), ("randomness", ctypes.c_float), ("step_cells", ctypes.c_float),
        ("tan_alpha", ctypes.c_float), ("flags", ctypes.c_uint32),
    ]


def make_params(mu=0.2, xi=2000.0, flow_height=1.0, persistence=0.9, randomness=0.16, step_cells=1.0,
                tan_alpha=-1.0) -> OracleParams:
    return OracleParams(mu, xi, flow_height, persistence, randomness, step_cells, tan_alpha, 0)


_libs: dict = {}


def _lib(prec: str):
    if prec not in _libs:
        # AVL_ORACLE_LIBDIR: load the twins from another directory (the sanitizer build of the tests)
        libdir = os.environ.get("AVL_ORACLE_LIBDIR")
        path = os.path.join(libdir or _HERE, f"liboracle_{prec}.so")
        if not libdir and not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        _libs[prec] = lib
    return _libs[prec]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _real(prec: str):
    return np.float32 if prec == "f32" else np.float64


def philox(ctr, key, prec: str = "f32") -> np.ndarray:
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    getattr(_lib(prec), f"oracle_philox4x32_10_{prec}")(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(dem: np.ndarray, cell_size: float, prec: str = "f32") -> np.ndarray:
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    h, w = dem.shape
    out = np.zeros((h, w, 4), dtype=_real(prec))
    getattr(_lib(prec), f"oracle_normals_{prec}")(_ptr(dem), ctypes.c_int(h), ctypes.c_int(w),
                                                  ctypes.c_float(cell_size), _ptr(out))
    return out


def release_mask(nrm: np.ndarray, dem: np.ndarray, smin: float, smax: float, zmin: float, zmax: float,
                 prec: str = "f32") -> np.ndarray:
    nrm = np.ascontiguousarray(nrm, dtype=_real(prec))
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    h, w = dem.shape
    out = np.zeros((h, w), dtype=np.uint8)
    getattr(_lib(prec), f"oracle_release_mask_{prec}")(
        _ptr(nrm), _ptr(dem), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_float(smin), ctypes.c_float(smax),
        ctypes.c_float(zmin), ctypes.c_float(zmax), _ptr(out))
    return out


def release_mask_fine(nrm: np.ndarray, dem: np.ndarray, mult: int, smin: float, smax: float, zmin: float,
                      zmax: float, prec: str = "f32") -> np.ndarray:
    """Release map at mult x mult texels per DEM cell: uint8 (mult*H, mult*W)."""
    nrm = np.ascontiguousarray(nrm, dtype=_real(prec))
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    h, w = dem.shape
    out = np.zeros((h * mult, w * mult), dtype=np.uint8)
    getattr(_lib(prec), f"oracle_release_mask_fine_{prec}")(
        _ptr(nrm), _ptr(dem), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_int(mult), ctypes.c_float(smin),
        ctypes.c_float(smax), ctypes.c_float(zmin), ctypes.c_float(zmax), _ptr(out))
    return out


def snow_cover(nrm: np.ndarray, dem: np.ndarray, snow_line: float, alt_blend: float, max_slope: float,
               slope_blend: float, prec: str = "f32") -> np.ndarray:
    """Snow-cover alpha (H, W) in [0, 1]."""
    nrm = np.ascontiguousarray(nrm, dtype=_real(prec))
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    h, w = dem.shape
    out = np.zeros((h, w), dtype=_real(prec))
    getattr(_lib(prec), f"oracle_snow_cover_{prec}")(
        _ptr(nrm), _ptr(dem), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_float(snow_line), ctypes.c_float(alt_blend),
        ctypes.c_float(max_slope), ctypes.c_float(slope_blend), _ptr(out))
    return out


def compact(mask: np.ndarray) -> np.ndarray:
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = mask.shape
    out = np.zeros(h * w, dtype=np.int32)
    fn = _lib("f32").oracle_compact_f32
    fn.restype = ctypes.c_int64
    n = fn(_ptr(mask), ctypes.c_int(h), ctypes.c_int(w), _ptr(out))
    return out[:n].copy()


def mipmap_levels(h: int, w: int) -> int:
    """Levels of the overlay mipmap including the full-resolution one: halving (rounding up) until 1 x 1."""
    n, m = 1, max(h, w)
    while m > 1:
        m = (m + 1) // 2
        n += 1
    return n


def mipmap(counts: np.ndarray, vmax: np.ndarray):
    """Levels 1 .. L-1 of the overlay mipmap (section 3): [(counts u64, vmax f32), ...], each level
    halving the previous one (rounding up); counts of the up-to-4 covered cells add, speeds take the max."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    vmax = np.ascontiguousarray(vmax, dtype=np.float32)
    h, w = counts.shape
    L = mipmap_levels(h, w)
    dims = []
    hh, ww = h, w
    for _ in range(1, L):
        hh, ww = (hh + 1) // 2, (ww + 1) // 2
        dims.append((hh, ww))
    total = sum(a * b for a, b in dims)
    cp = np.zeros(max(total, 1), dtype=np.uint64)
    vp = np.zeros(max(total, 1), dtype=np.float32)
    fn = _lib("f32").oracle_mipmap_f32
    fn.restype = ctypes.c_int64
    n = fn(_ptr(counts), _ptr(vmax), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_int(L), _ptr(cp), _ptr(vp))
    assert n == total
    out, at = [], 0
    for a, b in dims:
        out.append((cp[at:at + a * b].reshape(a, b).copy(), vp[at:at + a * b].reshape(a, b).copy()))
        at += a * b
    return out


@dataclass
class RunResult:
    counts: np.ndarray
    vmax: np.ndarray
    steps: int
    n_exit: int
    n_stop: int
    n_limit: int


def trajectories(dem: np.ndarray, mask: np.ndarray, cell_size: float, params: OracleParams,
                 particles_per_cell: int, step_limit: int, seed: int, run: int = 0,
                 prec: str = "f32") -> RunResult:
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = dem.shape
    assert mask.shape == (h, w)
    counts = np.zeros((h, w), dtype=np.uint32)
    vmax = np.zeros((h, w), dtype=_real(prec))
    stats = np.zeros(4, dtype=np.uint64)
    getattr(_lib(prec), f"oracle_trajectories_{prec}")(
        _ptr(dem), _ptr(mask), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_float(cell_size),
        ctypes.byref(params), ctypes.c_uint32(particles_per_cell), ctypes.c_uint32(step_limit),
        ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(counts), _ptr(vmax), _ptr(stats))
    return RunResult(counts, vmax, int(stats[0]), int(stats[1]), int(stats[2]), int(stats[3]))


def trajectories_fine(dem: np.ndarray, mask: np.ndarray, mult: int, cell_size: float, params: OracleParams,
                      particles_per_cell: int, step_limit: int, seed: int, run: int = 0,
                      prec: str = "f32") -> RunResult:
    """Run from a release texture with mult x mult texels per DEM cell (mask (mult*H, mult*W)); the
    rasters are (H, W)."""
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = dem.shape
    assert mask.shape == (h * mult, w * mult)
    counts = np.zeros((h, w), dtype=np.uint32)
    vmax = np.zeros((h, w), dtype=_real(prec))
    stats = np.zeros(4, dtype=np.uint64)
    getattr(_lib(prec), f"oracle_trajectories_fine_{prec}")(
        _ptr(dem), _ptr(mask), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_int(mult), ctypes.c_float(cell_size),
        ctypes.byref(params), ctypes.c_uint32(particles_per_cell), ctypes.c_uint32(step_limit),
        ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(counts), _ptr(vmax), _ptr(stats))
    return RunResult(counts, vmax, int(stats[0]), int(stats[1]), int(stats[2]), int(stats[3]))


@dataclass
class Trace:
    rows: np.ndarray  # (n, 8): x, y, z, gx, gy, dx, dy, v2
    reason: int
    steps: int

    @property
    def x(self): return self.rows[:, 0]

    @property
    def y(self): return self.rows[:, 1]

    @property
    def z(self): return self.rows[:, 2]

    @property
    def v2(self): return self.rows[:, 7]


def trace(dem: np.ndarray, cell_size: float, params: OracleParams, r: int, c: int, replica: int,
          step_limit: int, seed: int, run: int = 0, prec: str = "f32", mult: int = 1) -> Trace:
    """Path of one particle: replica `replica` of release texel (r, c) of a release texture with mult x mult
    texels per DEM cell (mult = 1: DEM cell (r, c))."""
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    h, w = dem.shape
    buf = np.zeros((step_limit + 1, 8), dtype=_real(prec))
    reason = ctypes.c_int32(0)
    steps = ctypes.c_uint64(0)
    fn = getattr(_lib(prec), f"oracle_trace_fine_{prec}")
    fn.restype = ctypes.c_int64
    n = fn(_ptr(dem), ctypes.c_int(h), ctypes.c_int(w), ctypes.c_float(cell_size), ctypes.byref(params),
           ctypes.c_int(r), ctypes.c_int(c), ctypes.c_int(mult), ctypes.c_uint32(replica),
           ctypes.c_uint32(step_limit), ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(buf), ctypes.byref(reason),
           ctypes.byref(steps))
    return Trace(buf[:n].copy(), int(reason.value), int(steps.value))


@dataclass
class SmoothResult:
    dep_q: np.ndarray      # (H, W) int64 deposit in fixed point (units of 2^-24)
    dep: np.ndarray        # (H, W) unquantised deposit in the working precision
    vel_q: np.ndarray      # (H, W) int64 velocity splat (fixed point), zero unless requested
    vel: np.ndarray
    steps: int
    n_exit: int
    n_stop: int
    n_limit: int


def smooth_forward(dem, mask, cell_size, params: OracleParams, particles_per_cell, step_limit, seed, run=0,
                   mass=None, vel_splat=False, prec="f32") -> SmoothResult:
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = dem.shape
    m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float32)
    dep_q = np.zeros((h, w), np.int64)
    dep = np.zeros((h, w), _real(prec))
    vel_q = np.zeros((h, w), np.int64)
    vel = np.zeros((h, w), _real(prec))
    stats = np.zeros(4, np.uint64)
    getattr(_lib(prec), f"oracle_smooth_forward_{prec}")(
        _ptr(dem), _ptr(mask), None if m is None else _ptr(m), ctypes.c_int(h), ctypes.c_int(w),
        ctypes.c_float(cell_size), ctypes.byref(params), ctypes.c_uint32(particles_per_cell),
        ctypes.c_uint32(step_limit), ctypes.c_uint64(seed), ctypes.c_uint32(run), ctypes.c_int(1 if vel_splat else 0),
        _ptr(dep_q), _ptr(dep), _ptr(vel_q), _ptr(vel), _ptr(stats))
    return SmoothResult(dep_q, dep, vel_q, vel, int(stats[0]), int(stats[1]), int(stats[2]), int(stats[3]))


@dataclass
class SmoothGrad:
    dmu: float
    dxi: float
    dh: float
    dmass: np.ndarray            # (H, W) float64
    per_particle: np.ndarray     # (n_particles, 4): dmu, dxi, dh, sum gD w  (release order)


def smooth_backward(dem, mask, cell_size, params: OracleParams, particles_per_cell, step_limit, seed, grad_dep,
                    run=0, mass=None, prec="f32") -> SmoothGrad:
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    g = np.ascontiguousarray(grad_dep, dtype=np.float32)
    h, w = dem.shape
    m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float32)
    gp = np.zeros(3, np.float64)
    gm = np.zeros((h, w), np.float64)
    pp = np.zeros((int(mask.astype(bool).sum()) * particles_per_cell, 4), _real(prec))
    fn = getattr(_lib(prec), f"oracle_smooth_backward_{prec}")
    rc = fn(_ptr(dem), _ptr(mask), None if m is None else _ptr(m), ctypes.c_int(h), ctypes.c_int(w),
            ctypes.c_float(cell_size), ctypes.byref(params), ctypes.c_uint32(particles_per_cell),
            ctypes.c_uint32(step_limit), ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(g), _ptr(gp), _ptr(gm),
            _ptr(pp) if pp.size else None)
    assert rc == 0
    return SmoothGrad(float(gp[0]), float(gp[1]), float(gp[2]), gm, pp)


def smooth_tangent(dem, mask, cell_size, params: OracleParams, particles_per_cell, step_limit, seed, grad_dep,
                   run=0, mass=None) -> tuple[float, float, float]:
    """Forward-mode (mu, xi, h) gradient, binary64."""
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    g = np.ascontiguousarray(grad_dep, dtype=np.float32)
    h, w = dem.shape
    m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float32)
    gp = np.zeros(3, np.float64)
    rc = _lib("f64").oracle_smooth_tangent_f64(
        _ptr(dem), _ptr(mask), None if m is None else _ptr(m), ctypes.c_int(h), ctypes.c_int(w),
        ctypes.c_float(cell_size), ctypes.byref(params), ctypes.c_uint32(particles_per_cell),
        ctypes.c_uint32(step_limit), ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(g), _ptr(gp))
    assert rc == 0
    return float(gp[0]), float(gp[1]), float(gp[2])


def smooth_particles(dem, mask, cell_size, params: OracleParams, particles_per_cell, step_limit, seed, grad_dep,
                     run=0, mass=None, prec="f64"):
    """Per particle (release order): share of L = sum gD * D, end reason, steps completed."""
    dem = np.ascontiguousarray(dem, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    g = np.ascontiguousarray(grad_dep, dtype=np.float32)
    h, w = dem.shape
    m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float32)
    n = int(mask.astype(bool).sum()) * particles_per_cell
    Lp = np.zeros(n, np.float64)
    reason = np.zeros(n, np.int32)
    steps = np.zeros(n, np.int32)
    rc = getattr(_lib(prec), f"oracle_smooth_particles_{prec}")(
        _ptr(dem), _ptr(mask), None if m is None else _ptr(m), ctypes.c_int(h), ctypes.c_int(w),
        ctypes.c_float(cell_size), ctypes.byref(params), ctypes.c_uint32(particles_per_cell),
        ctypes.c_uint32(step_limit), ctypes.c_uint64(seed), ctypes.c_uint32(run), _ptr(g), _ptr(Lp), _ptr(reason),
        _ptr(steps))
    assert rc == 0
    return Lp, reason, steps


# ------------------------------------------------------------------------------------------ calibration loop
# Calibration of the friction parameters against a target deposit: gradient descent with Adam (Kingma and
# Ba, "Adam: a method for stochastic optimization", ICLR 2015, algorithm 1) on (mu, xi), each step taking
# the loss and its gradient from the smooth forward and its adjoint.

def deposit_of(dep_q: np.ndarray) -> np.ndarray:
    """The float deposit of a fixed-point raster: q * 2^-24 in binary64, rounded once to binary32."""
    return (dep_q.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def mse_grad(dep: np.ndarray, target: np.ndarray) -> tuple[float, np.ndarray]:
    """L = mean((D - T)^2) (binary64 sum of the binary32 differences squared) and dL/dD = c (D - T) with
    c = 2 / N rounded to binary32 and the product in binary32."""
    d = dep.astype(np.float32) - target.astype(np.float32)
    n = d.size
    c = np.float32(2.0) / np.float32(n)
    loss = float(np.sum(d.astype(np.float64) ** 2) / n)
    return loss, (c * d).astype(np.float32)


@dataclass
class AdamState:
    lr: tuple            # per-parameter step sizes
    beta1: float
    beta2: float
    eps: float
    m: list
    v: list
    b1t: float = 1.0     # beta1^t and beta2^t, kept as running products
    b2t: float = 1.0
    t: int = 0


def adam_init(lr, beta1=0.9, beta2=0.999, eps=1e-8) -> AdamState:
    """Adam state for len(lr) parameters; the decay rates and eps enter as binary32 values (as the C ABI
    passes them)."""
    f = lambda v: float(np.float32(v))  # noqa: E731
    return AdamState(tuple(f(x) for x in lr), f(beta1), f(beta2), f(eps), [0.0] * len(lr), [0.0] * len(lr))


def adam_step(s: AdamState, theta: list, grad: list) -> list:
    """One Adam update in binary64: m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2; bias-corrected
    m^ = m / (1 - b1^t), v^ = v / (1 - b2^t); theta <- theta - lr m^ / (sqrt(v^) + eps)."""
    s.t += 1
    s.b1t *= s.beta1
    s.b2t *= s.beta2
    out = []
    for i, (th, g) in enumerate(zip(theta, grad)):
        s.m[i] = s.beta1 * s.m[i] + (1.0 - s.beta1) * g
        s.v[i] = s.beta2 * s.v[i] + (1.0 - s.beta2) * (g * g)
        mh = s.m[i] / (1.0 - s.b1t)
        vh = s.v[i] / (1.0 - s.b2t)
        out.append(th - s.lr[i] * mh / (float(np.sqrt(vh)) + s.eps))
    return out


def calibrate(dem, mask, cell_size, base: dict, particles_per_cell, step_limit, seed, target, mu0, xi0, n_iters,
              lr=(0.005, 50.0), beta1=0.9, beta2=0.999, eps=1e-8, mu_min=0.0, xi_min=1.0, run=0, mass=None):
    """Adam on (mu, xi) against `target` (float32 (H, W)). Returns the history, one row per iteration:
    (loss, mu, xi, dL/dmu, dL/dxi) at the iterate before its update, and the final (mu, xi). The model
    sees mu and xi rounded to binary32; after each update they are clamped to mu >= mu_min, xi >= xi_min."""
    s = adam_init(lr, beta1, beta2, eps)
    mu, xi = float(mu0), float(xi0)
    mu_lo, xi_lo = float(np.float32(mu_min)), float(np.float32(xi_min))
    hist = []
    for _ in range(n_iters):
        p = make_params(**dict(base, mu=float(np.float32(mu)), xi=float(np.float32(xi))))
        fwd = smooth_forward(dem, mask, cell_size, p, particles_per_cell, step_limit, seed, run, mass=mass)
        loss, gD = mse_grad(deposit_of(fwd.dep_q), target)
        g = smooth_backward(dem, mask, cell_size, p, particles_per_cell, step_limit, seed, gD, run, mass=mass)
        hist.append((loss, mu, xi, g.dmu, g.dxi))
        mu, xi = adam_step(s, [mu, xi], [g.dmu, g.dxi])
        mu, xi = max(mu, mu_lo), max(xi, xi_lo)
    return np.array(hist, np.float64), (mu, xi)
