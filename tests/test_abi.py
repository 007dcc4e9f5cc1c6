"""CPU checks of the C ABI: the library loads, exports every entry point that include/avl.h declares,
and rejects bad arguments on the host before any GPU work (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "avl.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"AVL_API\s+[\w\s\*]+?\b(avl_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("avl_normals", "avl_release_mask", "avl_release_cells", "avl_trajectories", "avl_workspace_bytes",
              "avl_strerror", "avl_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    avl = pytest.importorskip("paper_2506_23364_amd")
    lib = ctypes.CDLL(avl.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2506_23364_amd as avl
    monkeypatch.setattr(avl, "LIB_PATH", str(tmp_path / "libavl.so"))
    with pytest.raises(ImportError):
        avl._load()


@pytest.fixture(scope="module")
def L():
    import paper_2506_23364_amd as avl
    return avl


FAKE = 0x100000  # never dereferenced: every case below fails the host checks first


def test_strerror_and_workspace_size(L):
    for code in (0, -1, -2, -3, 7):
        assert L.lib.avl_strerror(code)
    assert L.workspace_bytes(0, 5) == 0
    n = 2048 * 2048
    assert L.workspace_bytes(2048, 2048) >= 4 * n
    assert L.workspace_bytes(3, 5) >= 4 * 15


def _traj(L, **kw):
    a = dict(dem=FAKE, mask=FAKE, H=16, W=16, cs=10.0, params=L.Params.make(), P=4, S=10, seed=1, run=0,
             counts=FAKE, vmax=FAKE, stats=None, ws=FAKE, wsb=L.workspace_bytes(16, 16), stream=None)
    a.update(kw)
    p = a["params"]
    return L.lib.avl_trajectories(a["dem"], a["mask"], a["H"], a["W"], a["cs"], ctypes.byref(p) if p else None,
                                  a["P"], a["S"], a["seed"], a["run"], a["counts"], a["vmax"], a["stats"], a["ws"],
                                  a["wsb"], a["stream"])


@pytest.mark.parametrize("kw", [
    dict(dem=None), dict(mask=None), dict(counts=None), dict(vmax=None), dict(ws=None), dict(params=None),
    dict(H=0), dict(W=-3), dict(H=65536, W=65536), dict(cs=0.0), dict(cs=float("nan")), dict(P=0),
])
def test_trajectories_rejects_bad_arguments(L, kw):
    assert _traj(L, **kw) == L.AVL_EINVAL
    assert L.lib.avl_last_error()


@pytest.mark.parametrize("field,value", [
    ("mu", -0.1), ("mu", float("inf")), ("xi", 0.0), ("xi", float("nan")), ("flow_height", 0.0),
    ("persistence", 1.5), ("persistence", -0.01), ("randomness", -1.0), ("step_cells", 0.0),
    ("step_cells", 17.0), ("tan_alpha", float("nan")), ("flags", 1),
])
def test_trajectories_rejects_bad_params(L, field, value):
    p = L.Params.make()
    setattr(p, field, value)
    assert _traj(L, params=p) == L.AVL_EINVAL


def test_trajectories_workspace_too_small(L):
    assert _traj(L, wsb=L.workspace_bytes(16, 16) - 1) == L.AVL_ENOMEM


def test_terrain_calls_reject_bad_arguments(L):
    lib = L.lib
    assert lib.avl_normals(None, 4, 4, 10.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_normals(FAKE, 1, 4, 10.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_normals(FAKE, 4, 4, -1.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_normals(FAKE, 4, 4, 10.0, FAKE + 4, None) == L.AVL_EINVAL  # misaligned float4 output
    assert lib.avl_release_mask(FAKE, FAKE, 4, 4, 40.0, 30.0, 0.0, 1.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_release_mask(FAKE, FAKE, 4, 4, 30.0, 91.0, 0.0, 1.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_release_mask(FAKE, FAKE, 4, 4, 30.0, 45.0, float("nan"), 1.0, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_release_mask(None, FAKE, 4, 4, 30.0, 45.0, 0.0, 1.0, FAKE, None) == L.AVL_EINVAL
    nrm = lib.avl_normals_release_mask
    assert nrm(None, 4, 4, 10.0, 30.0, 45.0, 0.0, 1.0, FAKE, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 10.0, 30.0, 45.0, 0.0, 1.0, FAKE, None, None) == L.AVL_EINVAL
    assert nrm(FAKE, 1, 4, 10.0, 30.0, 45.0, 0.0, 1.0, FAKE, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 0.0, 30.0, 45.0, 0.0, 1.0, FAKE, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 10.0, 30.0, 45.0, 0.0, 1.0, FAKE + 4, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 10.0, 40.0, 30.0, 0.0, 1.0, FAKE, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 10.0, 30.0, 91.0, 0.0, 1.0, FAKE, FAKE, None) == L.AVL_EINVAL
    assert nrm(FAKE, 4, 4, 10.0, 30.0, 45.0, 0.0, float("nan"), FAKE, FAKE, None) == L.AVL_EINVAL
    assert lib.avl_release_cells(FAKE, 4, 4, FAKE, FAKE, FAKE, 10, None) == L.AVL_ENOMEM
    assert lib.avl_release_cells(None, 4, 4, FAKE, FAKE, FAKE, 1 << 20, None) == L.AVL_EINVAL


def test_batched_workspace_size_and_padded_limits(L):
    assert L.batched_workspace_bytes(64, 64, 0, 1, 1) == 0
    assert L.batched_workspace_bytes(64, 64, 1, 0, 1) == 0
    one = L.batched_workspace_bytes(64, 64, 1, 1, 1)
    two = L.batched_workspace_bytes(64, 64, 2, 1, 1)
    assert two - one >= 66 * 66 * 4 - 255  # one more padded tile (H + 2) x (W + 2) f32, regions 256-aligned
    # the single-run call rejects grids whose padded DEM needs byte offsets of 2^32 or more
    assert _traj(L, H=32768, W=32766) == -1


def test_kernel_timing_needs_a_timed_call(L):
    ms = ctypes.c_float(0.0)
    assert L.lib.avl_last_kernel_ms(None) == -1
    assert L.lib.avl_last_kernel_ms(ctypes.byref(ms)) == -1
    assert "no timed" in L.lib.avl_last_error().decode()


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (3, 5), (37, 53), (2048, 2048), (1, 100000), (8193, 3)])
def test_mipmap_level_count_and_size(L, shape):
    import oracle
    h, w = shape
    assert L.lib.avl_mipmap_levels(h, w) == oracle.mipmap_levels(h, w)
    cells, hh, ww = 0, h, w
    while hh > 1 or ww > 1:
        hh, ww = (hh + 1) // 2, (ww + 1) // 2
        cells += hh * ww
    assert L.lib.avl_mipmap_cells(h, w) == cells


def test_mipmap_rejects_bad_arguments(L):
    assert L.lib.avl_overlay_mipmap(None, FAKE, 4, 4, FAKE, FAKE, None) == -1
    assert L.lib.avl_overlay_mipmap(FAKE, FAKE, 0, 4, FAKE, FAKE, None) == -1
    assert L.lib.avl_mipmap_levels(0, 3) == 0 and L.lib.avl_mipmap_cells(3, 0) == 0


def test_fine_workspace_size(L):
    assert L.fine_workspace_bytes(16, 16, 1) == L.workspace_bytes(16, 16)
    assert L.fine_workspace_bytes(16, 16, 0) == 0 and L.fine_workspace_bytes(16, 16, 17) == 0
    assert L.fine_workspace_bytes(0, 16, 2) == 0
    # the texel list and start records grow with the number of release texels (mult^2 H W)
    assert L.fine_workspace_bytes(64, 64, 4) - L.workspace_bytes(64, 64) >= 15 * 64 * 64 * (4 + 32) - 3 * 256


def _traj_fine(L, **kw):
    a = dict(dem=FAKE, mask=FAKE, H=16, W=16, mult=2, cs=10.0, params=L.Params.make(), P=4, S=10, seed=1, run=0,
             counts=FAKE, vmax=FAKE, stats=None, ws=FAKE, wsb=L.fine_workspace_bytes(16, 16, 2), stream=None)
    a.update(kw)
    p = a["params"]
    return L.lib.avl_trajectories_fine(a["dem"], a["mask"], a["H"], a["W"], a["mult"], a["cs"],
                                       ctypes.byref(p) if p else None, a["P"], a["S"], a["seed"], a["run"],
                                       a["counts"], a["vmax"], a["stats"], a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("kw", [
    dict(dem=None), dict(mask=None), dict(counts=None), dict(vmax=None), dict(ws=None), dict(params=None),
    dict(mult=0), dict(mult=17), dict(H=0), dict(H=20000, W=20000, mult=3), dict(cs=0.0), dict(P=0),
    dict(H=2, W=(1 << 22) + 1, mult=2), dict(H=(1 << 23), W=1, mult=1),
])
def test_trajectories_fine_rejects_bad_arguments(L, kw):
    assert _traj_fine(L, **kw) == L.AVL_EINVAL
    assert L.lib.avl_last_error()


def test_trajectories_fine_small_workspace(L):
    assert _traj_fine(L, wsb=L.fine_workspace_bytes(16, 16, 2) - 1) == L.AVL_ENOMEM
    assert _traj_fine(L, wsb=L.workspace_bytes(16, 16)) == L.AVL_ENOMEM


@pytest.mark.parametrize("args", [
    dict(nrm=None), dict(dem=None), dict(mask=None), dict(mult=0), dict(mult=17), dict(H=0),
    dict(H=30000, W=30000, mult=2), dict(H=(1 << 22), W=2, mult=2), dict(nrm=FAKE + 4),
    dict(smin=50.0, smax=40.0), dict(smax=91.0),
    dict(zmin=float("nan")),
])
def test_release_mask_fine_rejects_bad_arguments(L, args):
    a = dict(nrm=FAKE, dem=FAKE, H=16, W=16, mult=2, smin=30.0, smax=45.0, zmin=0.0, zmax=1.0, mask=FAKE)
    a.update(args)
    rc = L.lib.avl_release_mask_fine(a["nrm"], a["dem"], a["H"], a["W"], a["mult"], a["smin"], a["smax"], a["zmin"],
                                     a["zmax"], a["mask"], None)
    assert rc == L.AVL_EINVAL
    assert L.lib.avl_last_error()


@pytest.mark.parametrize("args", [
    dict(nrm=None), dict(dem=None), dict(alpha=None), dict(H=0), dict(nrm=FAKE + 8), dict(line=float("nan")),
    dict(zb=-1.0), dict(zb=float("inf")), dict(smax=91.0), dict(sb=50.0, smax=40.0), dict(sb=-1.0),
])
def test_snow_cover_rejects_bad_arguments(L, args):
    a = dict(nrm=FAKE, dem=FAKE, H=16, W=16, line=1000.0, zb=100.0, smax=40.0, sb=5.0, alpha=FAKE)
    a.update(args)
    rc = L.lib.avl_snow_cover(a["nrm"], a["dem"], a["H"], a["W"], a["line"], a["zb"], a["smax"], a["sb"],
                              a["alpha"], None)
    assert rc == L.AVL_EINVAL
    assert L.lib.avl_last_error()


def _calib(L, **kw):
    a = dict(dem=FAKE, mask=FAKE, mass=None, H=16, W=16, cs=10.0, start=L.Params.make(), P=4, S=100, seed=1, run=0,
             cap=10, target=FAKE, iters=3, adam=L.Adam.make(), hist=FAKE, res=L.Params(), ws=FAKE,
             wsb=L.lib.avl_calibrate_workspace_bytes(16, 16, 10, 4, 100), stream=None)
    a.update(kw)
    return L.lib.avl_calibrate(a["dem"], a["mask"], a["mass"], a["H"], a["W"], a["cs"],
                               ctypes.byref(a["start"]) if a["start"] else None, a["P"], a["S"], a["seed"], a["run"],
                               a["cap"], a["target"], a["iters"], ctypes.byref(a["adam"]) if a["adam"] else None,
                               a["hist"], ctypes.byref(a["res"]) if a["res"] is not None else None, a["ws"], a["wsb"],
                               a["stream"])


def test_calibrate_workspace_size(L):
    assert L.lib.avl_calibrate_workspace_bytes(16, 16, 10, 4, 100) >= \
        L.smooth_workspace_bytes(16, 16, 10, 4, 100) + 16 * 16 * 20
    assert L.lib.avl_calibrate_workspace_bytes(0, 16, 10, 4, 100) == 0


@pytest.mark.parametrize("kw", [
    dict(dem=None), dict(target=None), dict(adam=None), dict(res=None), dict(ws=None), dict(start=None),
    dict(hist=None), dict(iters=-1), dict(H=0), dict(P=0), dict(cs=0.0),
])
def test_calibrate_rejects_bad_arguments(L, kw):
    assert _calib(L, **kw) == L.AVL_EINVAL
    assert L.lib.avl_last_error()


@pytest.mark.parametrize("field,value", [
    ("lr_mu", 0.0), ("lr_xi", float("inf")), ("beta1", 1.0), ("beta2", -0.1), ("eps", 0.0), ("mu_min", -1.0),
    ("xi_min", 0.0),
])
def test_calibrate_rejects_bad_adam(L, field, value):
    adam = L.Adam.make()
    setattr(adam, field, value)
    assert _calib(L, adam=adam) == L.AVL_EINVAL


def test_calibrate_small_workspace(L):
    assert _calib(L, wsb=L.lib.avl_calibrate_workspace_bytes(16, 16, 10, 4, 100) - 1) == L.AVL_ENOMEM


def _smooth(L, fn, **kw):
    a = dict(dem=FAKE, mask=FAKE, mass=None, H=16, W=16, cs=10.0, params=L.Params.make(), P=4, S=100, seed=1, run=0,
             cap=10, ws=FAKE, stream=None)
    a.update(kw)
    wsb = a.get("wsb", L.smooth_workspace_bytes(a["H"], a["W"], a["cap"], a["P"], a["S"]))
    p = ctypes.byref(a["params"])
    if fn == "smooth":
        return L.lib.avl_trajectories_smooth(a["dem"], a["mask"], a["mass"], a["H"], a["W"], a["cs"], p, a["P"],
                                             a["S"], a["seed"], a["run"], a["cap"], 0, FAKE, None, None, None, None,
                                             None, a["ws"], wsb, a["stream"])
    return L.lib.avl_trajectories_backward(a["dem"], a["mask"], a["mass"], a["H"], a["W"], a["cs"], p, a["P"], a["S"],
                                           a["seed"], a["run"], a["cap"], FAKE, FAKE, FAKE, None, a["ws"], wsb,
                                           a["stream"])


# The padded patch's row offset is formed with a 24-bit multiply, so every particle pass needs W + 2 < 2^24;
# the entry points require H, W < 2^23. A 3 x 2^24 grid passes every other size check.
WIDE = dict(H=3, W=1 << 24)


def test_wide_grid_rejected_by_every_particle_pass(L):
    assert _traj(L, **WIDE, wsb=L.workspace_bytes(3, 1 << 24)) == L.AVL_EINVAL
    assert "2^23" in L.lib.avl_last_error().decode()
    assert _smooth(L, "smooth", **WIDE) == L.AVL_EINVAL
    assert "2^23" in L.lib.avl_last_error().decode()
    assert _smooth(L, "backward", **WIDE) == L.AVL_EINVAL
    assert "2^23" in L.lib.avl_last_error().decode()
    assert _calib(L, **WIDE, wsb=L.lib.avl_calibrate_workspace_bytes(3, 1 << 24, 10, 4, 100)) == L.AVL_EINVAL
    assert "2^23" in L.lib.avl_last_error().decode()
    h, w = WIDE["H"], WIDE["W"]
    rc = L.lib.avl_trajectories_batched(FAKE, 1, FAKE, 1, h, w, 10.0, FAKE, 1, FAKE, 1, 4, 100, FAKE, FAKE, None,
                                        None, FAKE, L.batched_workspace_bytes(h, w, 1, 1, 1), None)
    assert rc == L.AVL_EINVAL
    assert "2^23" in L.lib.avl_last_error().decode()


def test_grid_just_below_the_width_limit_passes_the_size_checks(L):
    # 2 x (2^23 - 1): accepted by the size checks, so a too-small workspace is what the calls report
    h, w = 2, (1 << 23) - 1
    assert _smooth(L, "smooth", H=h, W=w, wsb=1) == L.AVL_ENOMEM
    rc = L.lib.avl_trajectories_batched(FAKE, 1, FAKE, 1, h, w, 10.0, FAKE, 1, FAKE, 1, 4, 100, FAKE, FAKE, None,
                                        None, FAKE, 1, None)
    assert rc == L.AVL_ENOMEM



def _noalloc(L, **kw):
    a = dict(dem=FAKE, mask=FAKE, H=16, W=16, cs=10.0, params=L.Params.make(), P=4, S=10, seed=1, run=0,
             counts=FAKE, vmax=FAKE, stats=None, stream=None)
    a.update(kw)
    p = a["params"]
    return L.lib.avl_trajectories_noalloc(a["dem"], a["mask"], a["H"], a["W"], a["cs"], ctypes.byref(p) if p else None,
                                          a["P"], a["S"], a["seed"], a["run"], a["counts"], a["vmax"], a["stats"],
                                          a["stream"])


def test_noalloc_scratch_size(L):
    assert L.lib.avl_noalloc_scratch_bytes() == 64 << 20
    # 1280^2 fits the scratch; 1296^2 needs more than it holds
    assert L.workspace_bytes(1280, 1280) <= L.lib.avl_noalloc_scratch_bytes() < L.workspace_bytes(1296, 1296)


@pytest.mark.parametrize("kw", [
    dict(dem=None), dict(mask=None), dict(counts=None), dict(vmax=None), dict(params=None), dict(H=0), dict(W=-3),
    dict(cs=0.0), dict(P=0), dict(params="bad_mu"), dict(H=3, W=1 << 24),
    dict(H=1296, W=1296), dict(H=4096, W=420),  # more scratch than the library holds
])
def test_noalloc_rejects_bad_arguments_before_touching_the_gpu(L, kw):
    if kw.get("params") == "bad_mu":
        kw["params"] = L.Params.make(mu=-1.0)
    assert _noalloc(L, **kw) == L.AVL_EINVAL
    assert L.lib.avl_last_error()


def _record(L, **kw):
    a = dict(dem=FAKE, mask=FAKE, H=16, W=16, cs=10.0, params=L.Params.make(), P=4, S=10, seed=1, run=0, first=0,
             n=8, offsets=None, stride=0, points=None, speeds=None, ends=FAKE, counts=FAKE, vmax=FAKE, stats=None,
             ws=FAKE, wsb=L.workspace_bytes(16, 16), stream=None)
    a.update(kw)
    p = a["params"]
    return L.lib.avl_trajectories_record(a["dem"], a["mask"], a["H"], a["W"], a["cs"], ctypes.byref(p) if p else None,
                                         a["P"], a["S"], a["seed"], a["run"], a["first"], a["n"], a["offsets"],
                                         a["stride"], a["points"], a["speeds"], a["ends"], a["counts"], a["vmax"],
                                         a["stats"], a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("kw", [
    dict(n=0), dict(ends=None), dict(points=FAKE), dict(speeds=FAKE), dict(first=2**64 - 4, n=8),
    dict(points=FAKE, stride=1 << 20, n=1 << 21), dict(dem=None), dict(P=0), dict(wsb=16), dict(H=3, W=1 << 24),
])
def test_record_rejects_bad_arguments(L, kw):
    assert _record(L, **kw) in (L.AVL_EINVAL, L.AVL_ENOMEM)
    assert L.lib.avl_last_error()


def test_variant_info(L):
    n = L.tuning_variants()
    assert n >= 8
    shapes = set()
    for v in range(n):
        info = L.variant_info(v)
        assert info["block"] % 64 == 0 and info["table_slots"] % info["block"] == 0
        assert info["slots_per_lane"] >= 1 and info["waves_per_simd"] in (6, 8)
        shapes.add(tuple(info.values()))
    assert len(shapes) == n  # every candidate differs
    assert {L.variant_info(v)["block"] for v in range(n)} >= {512, 768, 1024}
    assert len({L.variant_info(v)["slots_per_lane"] for v in range(n)}) >= 3
    info = (ctypes.c_int32 * 8)()
    assert L.lib.avl_tuning_variant_info(n, ctypes.cast(info, ctypes.c_void_p)) == L.AVL_EINVAL
    assert L.lib.avl_tuning_variant_info(0, None) == L.AVL_EINVAL


def test_probe_switch_and_grid_query(L):
    assert L.lib.avl_set_probe(None, 0) == L.AVL_OK
    assert L.lib.avl_trajectory_grid(-1) == -1
    assert L.lib.avl_trajectory_grid(L.tuning_variants()) == -1


def test_smooth_tuning_override_range(L):
    nf, nb = L.smooth_tuning_variants()
    assert nf >= 2 and nb >= 2
    assert L.lib.avl_set_smooth_tuning(nf, 0) == L.AVL_EINVAL
    assert L.lib.avl_set_smooth_tuning(0, nb) == L.AVL_EINVAL
    assert L.lib.avl_set_smooth_tuning(-2, -1) == L.AVL_EINVAL
    assert L.lib.avl_set_smooth_tuning(nf - 1, nb - 1) == L.AVL_OK
    assert L.lib.avl_set_smooth_tuning(-1, -1) == L.AVL_OK
    assert L.lib.avl_smooth_tuning_variants(None, None) == L.AVL_EINVAL
