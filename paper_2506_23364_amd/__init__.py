"""MI355X-native hot path of the data-driven avalanche overlay (arXiv 2506.23364, section 5.2).

A thin binding over ``libavl.so`` (C ABI in ``include/avl.h``): it checks tensor types, allocates
outputs and workspace through PyTorch, passes device pointers and the current HIP stream, and turns
error codes into exceptions. Every step of the computation runs in the library's HIP kernels; there
is no CPU fallback. If the library is not built, importing this package raises ImportError.

Functions mirror the C entry points: :func:`normals`, :func:`release_mask`, :func:`release_cells`,
:func:`trajectories`; :func:`overlay` chains them (DEM -> normals -> release map -> trajectories).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = ["AvlError", "Params", "Run", "normals", "release_mask", "release_cells", "trajectories",
           "trajectories_batched", "trajectories_smooth", "trajectories_backward", "smooth_deposit", "SmoothDeposit",
           "overlay", "overlay_mipmap", "workspace_bytes", "batched_workspace_bytes", "smooth_workspace_bytes", "set_tuning",
           "tuning_variants", "last_variant", "LIB_PATH", "lib"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libavl.so")

AVL_OK, AVL_EINVAL, AVL_ENOMEM, AVL_EHIP = 0, -1, -2, -3


class AvlError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: error {code} ({detail})")
        self.code = code


class Params(ctypes.Structure):
    """Mirror of ``avl_params``."""
    _fields_ = [
        ("mu", ctypes.c_float), ("xi", ctypes.c_float), ("flow_height", ctypes.c_float),
        ("persistence", ctypes.c_float), ("randomness", ctypes.c_float), ("step_cells", ctypes.c_float),
        ("tan_alpha", ctypes.c_float), ("flags", ctypes.c_uint32),
    ]

    @classmethod
    def make(cls, mu=0.2, xi=2000.0, flow_height=1.0, persistence=0.9, randomness=0.16, step_cells=1.0,
             tan_alpha=-1.0, flags=0) -> "Params":
        return cls(mu, xi, flow_height, persistence, randomness, step_cells, tan_alpha, flags)


class Adam(ctypes.Structure):
    _fields_ = [("lr_mu", ctypes.c_float), ("lr_xi", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("mu_min", ctypes.c_float),
                ("xi_min", ctypes.c_float)]

    @classmethod
    def make(cls, lr_mu=0.003, lr_xi=30.0, beta1=0.9, beta2=0.999, eps=1e-8, mu_min=0.0, xi_min=1.0):
        return cls(lr_mu, lr_xi, beta1, beta2, eps, mu_min, xi_min)


class Run(ctypes.Structure):
    """Mirror of ``avl_run``: one run of a batch."""
    _fields_ = [("tile", ctypes.c_uint32), ("scenario", ctypes.c_uint32), ("param", ctypes.c_uint32),
                ("run_id", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2506_23364_amd/build.py` or "
                          "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, u64, f32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_float, ctypes.c_size_t)
    L.avl_normals.argtypes = [vp, i32, i32, f32, vp, vp]
    L.avl_release_mask.argtypes = [vp, vp, i32, i32, f32, f32, f32, f32, vp, vp]
    L.avl_normals_release_mask.argtypes = [vp, i32, i32, f32, f32, f32, f32, f32, vp, vp, vp]
    L.avl_workspace_bytes.argtypes = [i32, i32]
    L.avl_workspace_bytes.restype = sz
    L.avl_release_cells.argtypes = [vp, i32, i32, vp, vp, vp, sz, vp]
    L.avl_trajectories.argtypes = [vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, vp, vp, vp,
                                   vp, sz, vp]
    L.avl_trajectories_noalloc.argtypes = [vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, vp,
                                           vp, vp, vp]
    L.avl_trajectories_record.argtypes = [vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, u64, u32,
                                          vp, u32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.avl_trajectories_record.restype = ctypes.c_int
    L.avl_bench_schedule.argtypes = [i32, i32, i32, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp, vp]
    L.avl_bench_schedule.restype = ctypes.c_int
    L.avl_bench_gather.argtypes = [vp, i32, i32, vp, u64, vp, vp, sz, vp]
    L.avl_bench_gather.restype = ctypes.c_int
    L.avl_bench_atomics.argtypes = [i32, i32, vp, u64, vp, vp, vp]
    L.avl_bench_atomics.restype = ctypes.c_int
    L.avl_bench_stream.argtypes = [vp, vp, sz, vp]
    L.avl_bench_stream.restype = ctypes.c_int
    L.avl_noalloc_scratch_bytes.argtypes = []
    L.avl_noalloc_scratch_bytes.restype = sz
    L.avl_snow_cover.argtypes = [vp, vp, i32, i32, f32, f32, f32, f32, vp, vp]
    L.avl_release_mask_fine.argtypes = [vp, vp, i32, i32, i32, f32, f32, f32, f32, vp, vp]
    L.avl_fine_workspace_bytes.argtypes = [i32, i32, i32]
    L.avl_fine_workspace_bytes.restype = sz
    L.avl_trajectories_fine.argtypes = [vp, vp, i32, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, vp,
                                        vp, vp, vp, sz, vp]
    L.avl_mipmap_levels.argtypes = [i32, i32]
    L.avl_mipmap_levels.restype = i32
    L.avl_mipmap_cells.argtypes = [i32, i32]
    L.avl_mipmap_cells.restype = ctypes.c_int64
    L.avl_overlay_mipmap.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.avl_set_profiling.argtypes = [i32]
    L.avl_last_kernel_ms.argtypes = [ctypes.POINTER(ctypes.c_float)]
    L.avl_batched_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    L.avl_batched_workspace_bytes.restype = sz
    L.avl_trajectories_batched.argtypes = [vp, i32, vp, i32, i32, i32, f32, vp, i32, vp, i32, u32, u32, vp, vp, vp,
                                           vp, vp, sz, vp]
    L.avl_trajectories_batched.restype = ctypes.c_int
    L.avl_smooth_workspace_bytes.argtypes = [i32, i32, i32, u32, u32]
    L.avl_smooth_workspace_bytes.restype = sz
    L.avl_trajectories_smooth.argtypes = [vp, vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, i32,
                                          u32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.avl_trajectories_smooth.restype = ctypes.c_int
    L.avl_trajectories_backward.argtypes = [vp, vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32,
                                            i32, vp, vp, vp, vp, vp, sz, vp]
    L.avl_trajectories_backward.restype = ctypes.c_int
    L.avl_calibrate_workspace_bytes.argtypes = [i32, i32, i32, u32, u32]
    L.avl_calibrate_workspace_bytes.restype = sz
    L.avl_calibrate.argtypes = [vp, vp, vp, i32, i32, f32, ctypes.POINTER(Params), u32, u32, u64, u32, i32, vp, i32,
                                ctypes.POINTER(Adam), vp, ctypes.POINTER(Params), vp, sz, vp]
    L.avl_calibrate.restype = ctypes.c_int
    L.avl_set_tuning.argtypes = [i32, i32]
    L.avl_set_tuning.restype = ctypes.c_int
    L.avl_tuning_variants.argtypes = []
    L.avl_tuning_variants.restype = i32
    L.avl_set_smooth_tuning.argtypes = [i32, i32]
    L.avl_set_smooth_tuning.restype = ctypes.c_int
    L.avl_smooth_tuning_variants.argtypes = [vp, vp]
    L.avl_smooth_tuning_variants.restype = ctypes.c_int
    L.avl_tuning_variant_info.argtypes = [i32, vp]
    L.avl_tuning_variant_info.restype = ctypes.c_int
    L.avl_set_probe.argtypes = [vp, u64]
    L.avl_set_probe.restype = ctypes.c_int
    L.avl_trajectory_grid.argtypes = [i32]
    L.avl_trajectory_grid.restype = i32
    L.avl_last_variant.argtypes = []
    L.avl_last_variant.restype = i32
    L.avl_strerror.argtypes = [ctypes.c_int]
    L.avl_strerror.restype = ctypes.c_char_p
    L.avl_last_error.argtypes = []
    L.avl_last_error.restype = ctypes.c_char_p
    for name in ("avl_normals", "avl_release_mask", "avl_release_cells", "avl_trajectories", "avl_release_mask_fine",
                 "avl_trajectories_fine", "avl_snow_cover", "avl_trajectories_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(code: int, where: str) -> None:
    if code != AVL_OK:
        raise AvlError(code, where, (lib.avl_last_error() or b"").decode() or lib.avl_strerror(code).decode())


def _need(t: torch.Tensor, name: str, dtype: torch.dtype, dim: int | None = None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (there is no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dim is not None and t.dim() != dim:
        raise ValueError(f"{name} must have {dim} dimensions")


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


_ws: dict = {}


def _workspace(dev: torch.device, nbytes: int) -> torch.Tensor:
    """Per-device workspace, grown on demand and reused (calls on one stream are ordered)."""
    key = dev.index if dev.index is not None else torch.cuda.current_device()
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        _ws[key] = buf
    return buf


def workspace_bytes(h: int, w: int) -> int:
    return int(lib.avl_workspace_bytes(h, w))


def batched_workspace_bytes(h: int, w: int, n_tiles: int, n_masks: int, n_runs: int) -> int:
    return int(lib.avl_batched_workspace_bytes(h, w, n_tiles, n_masks, n_runs))


def set_tuning(variant: int = -1, graphs: bool = True) -> None:
    """variant -1 = autotune; graphs = capture batched calls into HIP graphs on non-null streams."""
    _check(lib.avl_set_tuning(variant, 1 if graphs else 0), "avl_set_tuning")


def tuning_variants() -> int:
    return int(lib.avl_tuning_variants())


def set_smooth_tuning(forward: int = -1, backward: int = -1) -> None:
    """Grid variants of the smooth forward and adjoint: -1 = the library's tuner, else a fixed index."""
    _check(lib.avl_set_smooth_tuning(forward, backward), "avl_set_smooth_tuning")


def smooth_tuning_variants() -> tuple[int, int]:
    nf, nb = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib.avl_smooth_tuning_variants(ctypes.byref(nf), ctypes.byref(nb)), "avl_smooth_tuning_variants")
    return int(nf.value), int(nb.value)


def variant_info(variant: int) -> dict:
    """Shape of a trajectory kernel variant."""
    info = (ctypes.c_int32 * 8)()
    _check(lib.avl_tuning_variant_info(variant, ctypes.cast(info, ctypes.c_void_p)), "avl_tuning_variant_info")
    keys = ("block", "iterations_per_epoch", "table_slots", "probes", "window", "retention", "waves_per_simd",
            "slots_per_lane")
    return dict(zip(keys, (int(v) for v in info)))


def set_probe(buf: "torch.Tensor | None") -> None:
    """Tail probe of later single-run trajectory calls: buf (uint64, 3 per block of the grid, zeroed by the
    caller) gets each block's start, slots-exhausted and end times on the GPU's 100 MHz clock; None stops it."""
    if buf is None:
        _check(lib.avl_set_probe(None, 0), "avl_set_probe")
        return
    _need(buf, "probe", torch.uint64, 1)
    _check(lib.avl_set_probe(buf.data_ptr(), buf.numel() // 3), "avl_set_probe")


def trajectory_grid(variant: int) -> int:
    return int(lib.avl_trajectory_grid(variant))


def last_variant() -> int:
    return int(lib.avl_last_variant())


def overlay_mipmap(counts: torch.Tensor, vmax: torch.Tensor):
    """Levels 1 .. L-1 of the overlay mipmap of (H, W) uint32 counts and float32 speeds: a list of
    (counts uint64, vmax float32) pairs, each level halving the previous one (rounding up)."""
    _need(counts, "counts", torch.uint32, 2)
    _need(vmax, "vmax", torch.float32, 2)
    h, w = counts.shape
    if tuple(vmax.shape) != (h, w):
        raise ValueError("counts and vmax must have the same shape")
    n = int(lib.avl_mipmap_cells(h, w))
    dev = counts.device
    cp = torch.empty(max(n, 1), dtype=torch.uint64, device=dev)
    vp = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.avl_overlay_mipmap(counts.data_ptr(), vmax.data_ptr(), h, w, cp.data_ptr(), vp.data_ptr(),
                                      _stream(dev)), "avl_overlay_mipmap")
    out, at = [], 0
    while h > 1 or w > 1:
        h, w = (h + 1) // 2, (w + 1) // 2
        out.append((cp[at:at + h * w].view(h, w), vp[at:at + h * w].view(h, w)))
        at += h * w
    return out


def set_profiling(enable: bool) -> None:
    """Time the trajectory kernel of later calls with HIP events on their stream (diagnostics)."""
    _check(lib.avl_set_profiling(1 if enable else 0), "avl_set_profiling")


def last_kernel_ms() -> float:
    """Duration of the trajectory kernel of the last timed call (waits for it)."""
    ms = ctypes.c_float(0.0)
    _check(lib.avl_last_kernel_ms(ctypes.byref(ms)), "avl_last_kernel_ms")
    return float(ms.value)


def normals(dem: torch.Tensor, cell_size: float) -> torch.Tensor:
    """(H, W) float32 DEM -> (H, W, 4) float32 (nx, ny, nz, slope degrees)."""
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    out = torch.empty((h, w, 4), dtype=torch.float32, device=dem.device)
    with torch.cuda.device(dem.device):
        _check(lib.avl_normals(dem.data_ptr(), h, w, cell_size, out.data_ptr(), _stream(dem.device)), "avl_normals")
    return out


def release_mask(nrm: torch.Tensor, dem: torch.Tensor, slope_min_deg: float, slope_max_deg: float,
                 z_min: float = float("-inf"), z_max: float = float("inf")) -> torch.Tensor:
    """Release map: uint8 (H, W), 1 where the steepness and elevation are in range."""
    _need(nrm, "normals", torch.float32, 3)
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    if nrm.shape != (h, w, 4):
        raise ValueError("normals must be (H, W, 4)")
    out = torch.empty((h, w), dtype=torch.uint8, device=dem.device)
    with torch.cuda.device(dem.device):
        _check(lib.avl_release_mask(nrm.data_ptr(), dem.data_ptr(), h, w, slope_min_deg, slope_max_deg, z_min, z_max,
                                    out.data_ptr(), _stream(dem.device)), "avl_release_mask")
    return out


def normals_release_mask(dem: torch.Tensor, cell_size: float, slope_min_deg: float, slope_max_deg: float,
                         z_min: float = float("-inf"), z_max: float = float("inf")) -> tuple[torch.Tensor, torch.Tensor]:
    """normals() and release_mask() of them in one pass: ((H, W, 4) float32 normals, (H, W) uint8 map)."""
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    nrm = torch.empty((h, w, 4), dtype=torch.float32, device=dem.device)
    mask = torch.empty((h, w), dtype=torch.uint8, device=dem.device)
    with torch.cuda.device(dem.device):
        _check(lib.avl_normals_release_mask(dem.data_ptr(), h, w, cell_size, slope_min_deg, slope_max_deg, z_min, z_max,
                                            nrm.data_ptr(), mask.data_ptr(), _stream(dem.device)),
               "avl_normals_release_mask")
    return nrm, mask


def release_cells(mask: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor]:
    """Row-major list of release texels: (cells int32 [H*W], n int32 [1]); cells[:n] are valid."""
    _need(mask, "mask", torch.uint8, 2)
    h, w = mask.shape
    cells = torch.empty(h * w, dtype=torch.int32, device=mask.device)
    n = torch.empty(1, dtype=torch.int32, device=mask.device)
    nb = workspace_bytes(h, w)
    with torch.cuda.device(mask.device):
        ws = _workspace(mask.device, nb)
        _check(lib.avl_release_cells(mask.data_ptr(), h, w, cells.data_ptr(), n.data_ptr(), ws.data_ptr(), ws.numel(),
                                     _stream(mask.device)), "avl_release_cells")
    return cells, n


@dataclass
class RunResult:
    counts: torch.Tensor   # (H, W) uint32: particle entries per texel
    vmax: torch.Tensor     # (H, W) float32: max speed per texel, m/s
    stats: torch.Tensor    # (4,) uint64: steps, exits, stops, step-limit ends


def trajectories(dem: torch.Tensor, mask: torch.Tensor, cell_size: float, params: Params,
                 particles_per_cell: int, step_limit: int, seed: int, run_id: int = 0,
                 out: RunResult | None = None) -> RunResult:
    """One pass of the trajectory model over every release texel of ``mask``."""
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    h, w = dem.shape
    if mask.shape != (h, w):
        raise ValueError("mask must have the DEM's shape")
    if out is None:
        out = RunResult(torch.empty((h, w), dtype=torch.uint32, device=dem.device),
                        torch.empty((h, w), dtype=torch.float32, device=dem.device),
                        torch.empty(4, dtype=torch.uint64, device=dem.device))
    nb = workspace_bytes(h, w)
    with torch.cuda.device(dem.device):
        ws = _workspace(dem.device, nb)
        _check(lib.avl_trajectories(dem.data_ptr(), mask.data_ptr(), h, w, cell_size, ctypes.byref(params),
                                    particles_per_cell, step_limit, seed & (2**64 - 1), run_id,
                                    out.counts.data_ptr(), out.vmax.data_ptr(), out.stats.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _stream(dem.device)), "avl_trajectories")
    return out


def trajectories_noalloc(dem: torch.Tensor, mask: torch.Tensor, cell_size: float, params: Params,
                         particles_per_cell: int, step_limit: int, seed: int, run_id: int = 0,
                         out: RunResult | None = None) -> RunResult:
    """:func:`trajectories` through the allocation-free entry point: the library works in its own per-GPU
    scratch instead of a workspace (the outputs are still the caller's; pass ``out`` to allocate nothing)."""
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    h, w = dem.shape
    if mask.shape != (h, w):
        raise ValueError("mask must have the DEM's shape")
    if out is None:
        out = RunResult(torch.empty((h, w), dtype=torch.uint32, device=dem.device),
                        torch.empty((h, w), dtype=torch.float32, device=dem.device),
                        torch.empty(4, dtype=torch.uint64, device=dem.device))
    with torch.cuda.device(dem.device):
        _check(lib.avl_trajectories_noalloc(dem.data_ptr(), mask.data_ptr(), h, w, cell_size, ctypes.byref(params),
                                            particles_per_cell, step_limit, seed & (2**64 - 1), run_id,
                                            out.counts.data_ptr(), out.vmax.data_ptr(), out.stats.data_ptr(),
                                            _stream(dem.device)), "avl_trajectories_noalloc")
    return out


@dataclass
class Paths:
    ends: torch.Tensor            # (n,) uint32: (accepted steps << 2) | end (0 limit, 1 exit, 2 stop); ~0 = none
    points: torch.Tensor | None   # (total, 2) float32 (x, y) in cell units, particle by particle
    speeds2: torch.Tensor | None  # (total,) float32 v^2 at each point
    offsets: torch.Tensor | None  # (n + 1,) int64: particle j's points are points[offsets[j]:offsets[j + 1]]
    run: RunResult


def _record_call(dem, mask, cell_size, params, P, S, seed, run_id, first, n, offsets, stride, points, speeds2, ends,
                 out):
    h, w = dem.shape
    nb = workspace_bytes(h, w)
    with torch.cuda.device(dem.device):
        ws = _workspace(dem.device, nb)
        _check(lib.avl_trajectories_record(dem.data_ptr(), mask.data_ptr(), h, w, cell_size, ctypes.byref(params), P, S,
                                           seed & (2**64 - 1), run_id, first, n,
                                           offsets.data_ptr() if offsets is not None else None, stride,
                                           points.data_ptr() if points is not None else None,
                                           speeds2.data_ptr() if speeds2 is not None else None, ends.data_ptr(),
                                           out.counts.data_ptr(), out.vmax.data_ptr(), out.stats.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _stream(dem.device)), "avl_trajectories_record")


def trajectory_paths(dem: torch.Tensor, mask: torch.Tensor, cell_size: float, params: Params, particles_per_cell: int,
                     step_limit: int, seed: int, run_id: int = 0, first: int = 0, n: int | None = None,
                     points: bool = True, speeds: bool = True) -> Paths:
    """Debug paths of particles [first, first + n) of a pass (n = None: to the last particle): one recording
    pass for the end records, then (points=True) a second one that writes every particle's points into a
    packed array sized from them. The rasters of the pass come with it."""
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    h, w = dem.shape
    if mask.shape != (h, w):
        raise ValueError("mask must have the DEM's shape")
    dev = dem.device
    if n is None:
        n = max(0, int(mask.count_nonzero().item()) * particles_per_cell - first)
    if n <= 0:
        raise ValueError("no particle in the recorded range")
    out = RunResult(torch.empty((h, w), dtype=torch.uint32, device=dev),
                    torch.empty((h, w), dtype=torch.float32, device=dev), torch.empty(4, dtype=torch.uint64, device=dev))
    ends = torch.empty(n, dtype=torch.uint32, device=dev)
    _record_call(dem, mask, cell_size, params, particles_per_cell, step_limit, seed, run_id, first, n, None, 0, None,
                 None, ends, out)
    if not points:
        return Paths(ends, None, None, None, out)
    e = ends.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    valid = e != 0xFFFFFFFF
    npts = torch.where(valid, (e >> 2) + 1 + ((e & 3) == 2).to(torch.int64), torch.zeros_like(e))
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    offsets[1:] = torch.cumsum(npts, 0)
    total = int(offsets[-1].item())
    pts = torch.empty((max(total, 1), 2), dtype=torch.float32, device=dev)
    sp = torch.empty(max(total, 1), dtype=torch.float32, device=dev) if speeds else None
    _record_call(dem, mask, cell_size, params, particles_per_cell, step_limit, seed, run_id, first, n, offsets, 0, pts,
                 sp, ends, out)
    return Paths(ends, pts[:total], sp[:total] if sp is not None else None, offsets, out)


@dataclass
class ReplaySchedule:
    gathers: torch.Tensor  # (n_gathers,) uint32 byte offsets of the 2 x 2 patches in the padded DEM, wave order
    visits: torch.Tensor   # (n_visits, 2) uint32 (cell, v^2 bits), wave order


def bench_schedule(shape, paths: Paths) -> ReplaySchedule:
    """The wave-order schedule of a recorded pass's gathers and cell visits (memory microbenchmarks)."""
    h, w = shape
    dev = paths.points.device
    n = paths.ends.numel()
    n_chunks = (n + 63) // 64
    totals = torch.zeros(2 * n_chunks, dtype=torch.int64, device=dev)
    args = (h, w, paths.points.data_ptr(), paths.speeds2.data_ptr(), paths.offsets.data_ptr(), paths.ends.data_ptr(), n)
    with torch.cuda.device(dev):
        _check(lib.avl_bench_schedule(0, *args, totals.data_ptr(), None, None, None, None, _stream(dev)),
               "avl_bench_schedule")
        t = totals.view(n_chunks, 2)
        base = torch.zeros((n_chunks + 1, 2), dtype=torch.int64, device=dev)
        base[1:] = torch.cumsum(t, 0)
        ng, nv = (int(v) for v in base[-1].tolist())
        gb = base[:-1, 0].contiguous()
        vb = base[:-1, 1].contiguous()
        gathers = torch.empty(max(ng, 1), dtype=torch.uint32, device=dev)
        visits = torch.empty((max(nv, 1), 2), dtype=torch.uint32, device=dev)
        _check(lib.avl_bench_schedule(1, *args, None, gb.data_ptr(), vb.data_ptr(), gathers.data_ptr(),
                                      visits.data_ptr(), _stream(dev)), "avl_bench_schedule")
    return ReplaySchedule(gathers[:ng], visits[:nv])


def bench_gather(dem: torch.Tensor, sched: ReplaySchedule) -> torch.Tensor:
    """Replay of the gathers of a schedule (memory microbenchmark); returns the device checksum."""
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    chk = torch.empty(1, dtype=torch.uint32, device=dem.device)
    with torch.cuda.device(dem.device):
        ws = _workspace(dem.device, workspace_bytes(h, w))
        _check(lib.avl_bench_gather(dem.data_ptr(), h, w, sched.gathers.data_ptr(), sched.gathers.numel(),
                                    chk.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dem.device)), "avl_bench_gather")
    return chk


def bench_atomics(shape, sched: ReplaySchedule, out: tuple | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """Replay of the cell visits of a schedule as unaggregated raster atomics: (counts, v^2 max bits)."""
    h, w = shape
    dev = sched.visits.device
    counts, bits = out if out is not None else (torch.empty((h, w), dtype=torch.uint32, device=dev),
                                                torch.empty((h, w), dtype=torch.uint32, device=dev))
    with torch.cuda.device(dev):
        _check(lib.avl_bench_atomics(h, w, sched.visits.data_ptr(), sched.visits.shape[0], counts.data_ptr(),
                                     bits.data_ptr(), _stream(dev)), "avl_bench_atomics")
    return counts, bits


def bench_stream(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Device copy of src into dst (same byte size, a multiple of 16): the HBM stream microbenchmark."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size")
    with torch.cuda.device(src.device):
        _check(lib.avl_bench_stream(src.data_ptr(), dst.data_ptr(), nbytes, _stream(src.device)), "avl_bench_stream")


def snow_cover(nrm: torch.Tensor, dem: torch.Tensor, snow_line: float, alt_blend: float, max_slope_deg: float,
               slope_blend_deg: float) -> torch.Tensor:
    """Snow-cover alpha: float32 (H, W) in [0, 1]."""
    _need(nrm, "normals", torch.float32, 3)
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    if nrm.shape != (h, w, 4):
        raise ValueError("normals must be (H, W, 4)")
    out = torch.empty((h, w), dtype=torch.float32, device=dem.device)
    with torch.cuda.device(dem.device):
        _check(lib.avl_snow_cover(nrm.data_ptr(), dem.data_ptr(), h, w, snow_line, alt_blend, max_slope_deg,
                                  slope_blend_deg, out.data_ptr(), _stream(dem.device)), "avl_snow_cover")
    return out


def fine_workspace_bytes(h: int, w: int, mult: int) -> int:
    return int(lib.avl_fine_workspace_bytes(h, w, mult))


def release_mask_fine(nrm: torch.Tensor, dem: torch.Tensor, mult: int, slope_min_deg: float, slope_max_deg: float,
                      z_min: float = float("-inf"), z_max: float = float("inf")) -> torch.Tensor:
    """Release map at mult x mult texels per DEM cell: uint8 (mult*H, mult*W)."""
    _need(nrm, "normals", torch.float32, 3)
    _need(dem, "dem", torch.float32, 2)
    h, w = dem.shape
    if nrm.shape != (h, w, 4):
        raise ValueError("normals must be (H, W, 4)")
    out = torch.empty((h * mult, w * mult), dtype=torch.uint8, device=dem.device)
    with torch.cuda.device(dem.device):
        _check(lib.avl_release_mask_fine(nrm.data_ptr(), dem.data_ptr(), h, w, mult, slope_min_deg, slope_max_deg,
                                         z_min, z_max, out.data_ptr(), _stream(dem.device)), "avl_release_mask_fine")
    return out


def trajectories_fine(dem: torch.Tensor, mask: torch.Tensor, mult: int, cell_size: float, params: Params,
                      particles_per_cell: int, step_limit: int, seed: int, run_id: int = 0,
                      out: RunResult | None = None) -> RunResult:
    """One pass from a release texture with mult x mult texels per DEM cell (mask (mult*H, mult*W)); the
    rasters have the DEM's shape."""
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    h, w = dem.shape
    if mask.shape != (h * mult, w * mult):
        raise ValueError("mask must be (mult*H, mult*W)")
    if out is None:
        out = RunResult(torch.empty((h, w), dtype=torch.uint32, device=dem.device),
                        torch.empty((h, w), dtype=torch.float32, device=dem.device),
                        torch.empty(4, dtype=torch.uint64, device=dem.device))
    nb = fine_workspace_bytes(h, w, mult)
    if nb == 0:
        raise ValueError("mult out of range")
    with torch.cuda.device(dem.device):
        ws = _workspace(dem.device, nb)
        _check(lib.avl_trajectories_fine(dem.data_ptr(), mask.data_ptr(), h, w, mult, cell_size, ctypes.byref(params),
                                         particles_per_cell, step_limit, seed & (2**64 - 1), run_id,
                                         out.counts.data_ptr(), out.vmax.data_ptr(), out.stats.data_ptr(),
                                         ws.data_ptr(), ws.numel(), _stream(dem.device)), "avl_trajectories_fine")
    return out


def params_tensor(params, device) -> torch.Tensor:
    """Device array of avl_params from a list of Params (or dicts of Params.make keywords)."""
    ps = [p if isinstance(p, Params) else Params.make(**p) for p in params]
    raw = b"".join(bytes(p) for p in ps)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


def runs_tensor(runs, device) -> torch.Tensor:
    """Device array of avl_run from a list of Run (or (tile, scenario, param, run_id, seed) tuples)."""
    rs = [r if isinstance(r, Run) else Run(*r) for r in runs]
    raw = b"".join(bytes(r) for r in rs)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


@dataclass
class BatchResult:
    counts: torch.Tensor   # (n_runs, H, W) uint32
    vmax: torch.Tensor     # (n_runs, H, W) float32
    stats: torch.Tensor    # (n_runs, 4) uint64
    status: torch.Tensor   # (n_runs,) int32: 0 ran, 1 bad index, 2 bad parameters


def trajectories_batched(dems: torch.Tensor, masks: torch.Tensor, cell_size: float, params: torch.Tensor,
                         runs: torch.Tensor, particles_per_cell: int, step_limit: int,
                         out: BatchResult | None = None) -> BatchResult:
    """Many runs in one launch. dems (n_tiles, H, W) f32; masks (n_masks, H, W) u8; params and runs are
    device byte tensors from params_tensor / runs_tensor (they may be rewritten between calls)."""
    _need(dems, "dems", torch.float32, 3)
    _need(masks, "masks", torch.uint8, 3)
    _need(params, "params", torch.uint8, 1)
    _need(runs, "runs", torch.uint8, 1)
    n_tiles, h, w = dems.shape
    n_masks = masks.shape[0]
    if masks.shape[1:] != (h, w):
        raise ValueError("masks must have the tiles' shape")
    n_params = params.numel() // ctypes.sizeof(Params)
    n_runs = runs.numel() // ctypes.sizeof(Run)
    if out is None:
        dev = dems.device
        out = BatchResult(torch.empty((n_runs, h, w), dtype=torch.uint32, device=dev),
                          torch.empty((n_runs, h, w), dtype=torch.float32, device=dev),
                          torch.empty((n_runs, 4), dtype=torch.uint64, device=dev),
                          torch.empty(n_runs, dtype=torch.int32, device=dev))
    nb = batched_workspace_bytes(h, w, n_tiles, n_masks, n_runs)
    with torch.cuda.device(dems.device):
        ws = _workspace(dems.device, nb)
        _check(lib.avl_trajectories_batched(dems.data_ptr(), n_tiles, masks.data_ptr(), n_masks, h, w, cell_size,
                                            params.data_ptr(), n_params, runs.data_ptr(), n_runs, particles_per_cell,
                                            step_limit, out.counts.data_ptr(), out.vmax.data_ptr(),
                                            out.stats.data_ptr(), out.status.data_ptr(), ws.data_ptr(), ws.numel(),
                                            _stream(dems.device)), "avl_trajectories_batched")
    return out


def smooth_workspace_bytes(h: int, w: int, max_release_cells: int, particles_per_cell: int, step_limit: int) -> int:
    return int(lib.avl_smooth_workspace_bytes(h, w, max_release_cells, particles_per_cell, step_limit))


@dataclass
class SmoothRun:
    """Result of the smooth forward; `workspace` holds the checkpoints the adjoint needs."""
    deposit_q: torch.Tensor   # (H, W) int64, units of 2^-24
    deposit: torch.Tensor     # (H, W) float32
    velocity_q: torch.Tensor | None
    velocity: torch.Tensor | None
    stats: torch.Tensor       # (4,) uint64
    status: torch.Tensor      # (1,) int32: 0 ok, 3 more release cells than max_release_cells
    workspace: torch.Tensor
    max_release_cells: int


def trajectories_smooth(dem: torch.Tensor, mask: torch.Tensor, cell_size: float, params: Params,
                        particles_per_cell: int, step_limit: int, seed: int, run_id: int = 0,
                        mass: torch.Tensor | None = None, velocity: bool = False,
                        max_release_cells: int | None = None) -> SmoothRun:
    """Smooth forward: deposit of the released mass at each particle's resting point (own workspace)."""
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    h, w = dem.shape
    if mass is not None:
        _need(mass, "mass", torch.float32, 2)
    if max_release_cells is None:
        max_release_cells = int(mask.count_nonzero().item())
    dev = dem.device
    ws = torch.empty(max(256, smooth_workspace_bytes(h, w, max_release_cells, particles_per_cell, step_limit)),
                     dtype=torch.uint8, device=dev)
    dq = torch.empty((h, w), dtype=torch.int64, device=dev)
    df = torch.empty((h, w), dtype=torch.float32, device=dev)
    vq = torch.empty((h, w), dtype=torch.int64, device=dev) if velocity else None
    vf = torch.empty((h, w), dtype=torch.float32, device=dev) if velocity else None
    stats = torch.empty(4, dtype=torch.uint64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.avl_trajectories_smooth(dem.data_ptr(), mask.data_ptr(), mass.data_ptr() if mass is not None else None,
                                           h, w, cell_size, ctypes.byref(params), particles_per_cell, step_limit,
                                           seed & (2**64 - 1), run_id, max_release_cells, 1 if velocity else 0,
                                           dq.data_ptr(), df.data_ptr(), vq.data_ptr() if velocity else None,
                                           vf.data_ptr() if velocity else None, stats.data_ptr(), status.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _stream(dev)), "avl_trajectories_smooth")
    return SmoothRun(dq, df, vq, vf, stats, status, ws, max_release_cells)


def trajectories_backward(run: SmoothRun, dem: torch.Tensor, mask: torch.Tensor, cell_size: float, params: Params,
                          particles_per_cell: int, step_limit: int, seed: int, grad_deposit: torch.Tensor,
                          run_id: int = 0, mass: torch.Tensor | None = None, per_particle: bool = False):
    """Adjoint of `run`'s deposit: (dparams float64 [dmu, dxi, dh], dmass (H, W), per-particle or None)."""
    _need(grad_deposit, "grad_deposit", torch.float32, 2)
    h, w = dem.shape
    dev = dem.device
    dparams = torch.empty(3, dtype=torch.float64, device=dev)
    dmass = torch.empty((h, w), dtype=torch.float32, device=dev)
    pp = (torch.empty((4, run.max_release_cells * particles_per_cell), dtype=torch.float32, device=dev)
          if per_particle else None)
    with torch.cuda.device(dev):
        _check(lib.avl_trajectories_backward(dem.data_ptr(), mask.data_ptr(),
                                             mass.data_ptr() if mass is not None else None, h, w, cell_size,
                                             ctypes.byref(params), particles_per_cell, step_limit, seed & (2**64 - 1),
                                             run_id, run.max_release_cells, grad_deposit.data_ptr(), dparams.data_ptr(),
                                             dmass.data_ptr(), pp.data_ptr() if pp is not None else None,
                                             run.workspace.data_ptr(), run.workspace.numel(), _stream(dev)),
               "avl_trajectories_backward")
    return dparams, dmass, pp


def calibrate(dem: torch.Tensor, mask: torch.Tensor, cell_size: float, start: Params, particles_per_cell: int,
              step_limit: int, seed: int, target: torch.Tensor, n_iters: int, adam: Adam | None = None,
              run_id: int = 0, mass: torch.Tensor | None = None, max_release_cells: int | None = None):
    """Adam on (mu, xi) against `target`: (history float64 (n_iters, 5) of (L, mu, xi, dL/dmu, dL/dxi) per
    iterate, final Params)."""
    import numpy as np
    _need(dem, "dem", torch.float32, 2)
    _need(mask, "mask", torch.uint8, 2)
    _need(target, "target", torch.float32, 2)
    h, w = dem.shape
    if mass is not None:
        _need(mass, "mass", torch.float32, 2)
    if max_release_cells is None:
        max_release_cells = int(mask.count_nonzero().item())
    adam = adam or Adam.make()
    nb = int(lib.avl_calibrate_workspace_bytes(h, w, max_release_cells, particles_per_cell, step_limit))
    hist = np.zeros((max(n_iters, 1), 5), np.float64)
    result = Params()
    with torch.cuda.device(dem.device):
        ws = _workspace(dem.device, max(nb, 256))
        _check(lib.avl_calibrate(dem.data_ptr(), mask.data_ptr(), mass.data_ptr() if mass is not None else None, h, w,
                                 cell_size, ctypes.byref(start), particles_per_cell, step_limit, seed & (2**64 - 1),
                                 run_id, max_release_cells, target.data_ptr(), n_iters, ctypes.byref(adam),
                                 hist.ctypes.data_as(ctypes.c_void_p), ctypes.byref(result), ws.data_ptr(), ws.numel(),
                                 _stream(dem.device)), "avl_calibrate")
    return hist[:n_iters], result


class SmoothDeposit(torch.autograd.Function):
    """deposit = f(mu, xi, h, mass): forward = smooth pass, backward = the adjoint kernel."""

    @staticmethod
    def forward(ctx, mu, xi, h, mass, dem, mask, cell_size, base, particles_per_cell, step_limit, seed, run_id,
                max_release_cells):
        params = Params.make(**dict(base, mu=float(mu), xi=float(xi), flow_height=float(h)))
        run = trajectories_smooth(dem, mask, cell_size, params, particles_per_cell, step_limit, seed, run_id,
                                  mass=mass.detach().contiguous(), max_release_cells=max_release_cells)
        ctx.run, ctx.params = run, params
        ctx.args = (dem, mask, cell_size, particles_per_cell, step_limit, seed, run_id)
        ctx.save_for_backward(mass)
        return run.deposit

    @staticmethod
    def backward(ctx, grad_dep):
        (mass,) = ctx.saved_tensors
        dem, mask, cell_size, P, S, seed, run_id = ctx.args
        dparams, dmass, _ = trajectories_backward(ctx.run, dem, mask, cell_size, ctx.params, P, S, seed,
                                                  grad_dep.contiguous().float(), run_id, mass.detach().contiguous())
        dp = dparams.float()
        return (dp[0], dp[1], dp[2], dmass, None, None, None, None, None, None, None, None, None)


def smooth_deposit(mu: torch.Tensor, xi: torch.Tensor, h: torch.Tensor, mass: torch.Tensor, dem: torch.Tensor,
                   mask: torch.Tensor, cell_size: float, particles_per_cell: int, step_limit: int, seed: int,
                   run_id: int = 0, persistence: float = 0.9, randomness: float = 0.16, step_cells: float = 1.0,
                   max_release_cells: int | None = None) -> torch.Tensor:
    """Differentiable deposit raster (float32 (H, W)) with gradients to mu, xi, h (0-d tensors) and mass."""
    base = dict(persistence=persistence, randomness=randomness, step_cells=step_cells, tan_alpha=-1.0)
    return SmoothDeposit.apply(mu, xi, h, mass, dem, mask, cell_size, base, particles_per_cell, step_limit, seed,
                               run_id, max_release_cells)


def overlay(dem: torch.Tensor, cell_size: float, slope_min_deg: float, slope_max_deg: float, z_min: float,
            z_max: float, params: Params, particles_per_cell: int, step_limit: int, seed: int,
            run_id: int = 0) -> tuple[torch.Tensor, torch.Tensor, RunResult]:
    """The whole avalanche overlay: normals -> release map -> trajectories."""
    nrm = normals(dem, cell_size)
    mask = release_mask(nrm, dem, slope_min_deg, slope_max_deg, z_min, z_max)
    return nrm, mask, trajectories(dem, mask, cell_size, params, particles_per_cell, step_limit, seed, run_id)
