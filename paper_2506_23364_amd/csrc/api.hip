// extern "C" entry points of libavl.so: host-side argument checks, derived constants, workspace
// carving and kernel enqueueing. See include/avl.h for the contract of each call.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/avl.h"
#include "avl_internal.h"

namespace avl {

size_t workspace_bytes(int64_t n) {
    return 256 + round256((size_t)scan_blocks(n) * sizeof(uint32_t)) + round256((size_t)n * sizeof(int32_t)) +
           2 * round256((size_t)kXcds * n * sizeof(uint32_t));
}

Workspace carve(void* base, int64_t n) {
    char* p = static_cast<char*>(base);
    Workspace w;
    w.n_cells = reinterpret_cast<int32_t*>(p);
    w.stats = reinterpret_cast<unsigned long long*>(p + 16);
    w.queues = reinterpret_cast<unsigned long long*>(p + 64);
    p += 256;
    w.blk = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)scan_blocks(n) * sizeof(uint32_t));
    w.cells = reinterpret_cast<int32_t*>(p);
    p += round256((size_t)n * sizeof(int32_t));
    w.priv_counts = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)kXcds * n * sizeof(uint32_t));
    w.priv_vmax2 = reinterpret_cast<uint32_t*>(p);
    return w;
}

}  // namespace avl

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, const char* detail = nullptr) {
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, detail ? detail : "");
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    g_last_error = buf;
    return AVL_EHIP;
}

bool grid_ok(int32_t H, int32_t W, int32_t min_dim) {
    return H >= min_dim && W >= min_dim && (int64_t)H * (int64_t)W < (int64_t(1) << 31);
}

bool finite(float v) { return std::isfinite(v); }

const char* check_params(const avl_params* p) {
    if (!p) return "params is NULL";
    if (!finite(p->mu) || p->mu < 0.0f) return "mu must be finite and >= 0";
    if (std::isnan(p->xi) || !(p->xi > 0.0f)) return "xi must be > 0 (+inf allowed)";
    if (!finite(p->flow_height) || !(p->flow_height > 0.0f)) return "flow_height must be finite and > 0";
    if (!(p->persistence >= 0.0f && p->persistence <= 1.0f)) return "persistence must be in [0, 1]";
    if (!finite(p->randomness) || p->randomness < 0.0f) return "randomness must be finite and >= 0";
    if (!finite(p->step_cells) || !(p->step_cells > 0.0f) || p->step_cells > 16.0f)
        return "step_cells must be in (0, 16]";
    if (!finite(p->tan_alpha)) return "tan_alpha must be finite";
    if (p->flags != 0u) return "flags must be 0";
    return nullptr;
}

}  // namespace

extern "C" {

const char* avl_strerror(int code) {
    switch (code) {
        case AVL_OK: return "AVL_OK: success";
        case AVL_EINVAL: return "AVL_EINVAL: invalid argument";
        case AVL_ENOMEM: return "AVL_ENOMEM: workspace too small";
        case AVL_EHIP: return "AVL_EHIP: HIP runtime error";
        default: return "unknown avl error code";
    }
}

const char* avl_last_error(void) { return g_last_error.c_str(); }

size_t avl_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    return avl::workspace_bytes((int64_t)H * W);
}

int avl_normals(const float* dem, int32_t H, int32_t W, float cell_size, float* normals4, void* stream) {
    g_last_error.clear();
    if (!dem || !normals4) return fail(AVL_EINVAL, "avl_normals: null pointer");
    if (!grid_ok(H, W, 2)) return fail(AVL_EINVAL, "avl_normals: need H, W >= 2 and H*W < 2^31");
    if (!finite(cell_size) || !(cell_size > 0.0f)) return fail(AVL_EINVAL, "avl_normals: cell_size must be > 0");
    if (reinterpret_cast<uintptr_t>(normals4) & 15) return fail(AVL_EINVAL, "avl_normals: normals4 not 16-byte aligned");
    hipError_t e = avl::launch_normals(dem, H, W, cell_size, normals4, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_normals");
}

int avl_release_mask(const float* normals4, const float* dem, int32_t H, int32_t W, float slope_min_deg,
                     float slope_max_deg, float z_min, float z_max, uint8_t* mask, void* stream) {
    g_last_error.clear();
    if (!normals4 || !dem || !mask) return fail(AVL_EINVAL, "avl_release_mask: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_release_mask: need H, W >= 1 and H*W < 2^31");
    if (reinterpret_cast<uintptr_t>(normals4) & 15)
        return fail(AVL_EINVAL, "avl_release_mask: normals4 not 16-byte aligned");
    if (!(slope_min_deg >= 0.0f && slope_min_deg <= slope_max_deg && slope_max_deg <= 90.0f))
        return fail(AVL_EINVAL, "avl_release_mask: need 0 <= slope_min_deg <= slope_max_deg <= 90");
    if (std::isnan(z_min) || std::isnan(z_max)) return fail(AVL_EINVAL, "avl_release_mask: NaN elevation bound");
    const double d2r = 3.14159265358979323846 / 180.0;
    const float cmin = (float)std::cos((double)slope_max_deg * d2r);
    const float cmax = (float)std::cos((double)slope_min_deg * d2r);
    hipError_t e = avl::launch_release_mask(normals4, dem, (int64_t)H * W, cmin, cmax, z_min, z_max, mask,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_release_mask");
}

int avl_release_cells(const uint8_t* mask, int32_t H, int32_t W, int32_t* cells, int32_t* n_cells,
                      void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!mask || !cells || !n_cells || !workspace) return fail(AVL_EINVAL, "avl_release_cells: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_release_cells: need H, W >= 1 and H*W < 2^31");
    const int64_t n = (int64_t)H * W;
    if (workspace_bytes < avl::workspace_bytes(n)) return fail(AVL_ENOMEM, "avl_release_cells: workspace too small");
    avl::Workspace ws = avl::carve(workspace, n);
    hipError_t e = avl::launch_compact(mask, n, cells, n_cells, ws.blk, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_release_cells");
}

int avl_trajectories(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                     const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                     uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                     size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!dem || !mask || !counts || !vmax || !workspace) return fail(AVL_EINVAL, "avl_trajectories: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_trajectories: need H, W >= 1 and H*W < 2^31");
    if (!finite(cell_size) || !(cell_size > 0.0f)) return fail(AVL_EINVAL, "avl_trajectories: cell_size must be > 0");
    if (particles_per_cell == 0) return fail(AVL_EINVAL, "avl_trajectories: particles_per_cell must be >= 1");
    if (const char* why = check_params(params)) return fail(AVL_EINVAL, "avl_trajectories: %s", why);
    const int64_t n = (int64_t)H * W;
    if (workspace_bytes < avl::workspace_bytes(n)) return fail(AVL_ENOMEM, "avl_trajectories: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::Workspace ws = avl::carve(workspace, n);

    // derived constants, binary32, in this order
    avl::TrajArgs a{};
    const float g = 9.81f;
    a.g2 = g + g;
    a.per = params->persistence;
    a.Q = 1.0f - a.per;
    a.rnd = params->randomness;
    a.L = params->step_cells;
    const float dl = a.L * cell_size;
    a.dl2 = dl * dl;
    a.mdl = params->mu * dl;
    a.cd = a.g2 / (params->xi * params->flow_height);
    a.use_alpha = params->tan_alpha >= 0.0f ? 1 : 0;
    a.tca = params->tan_alpha * cell_size;
    a.dem = dem;
    a.cells = ws.cells;
    a.n_cells = ws.n_cells;
    a.queues = ws.queues;
    a.counts = ws.priv_counts;
    a.vmax2 = ws.priv_vmax2;
    a.stats = stats ? reinterpret_cast<unsigned long long*>(stats) : ws.stats;
    a.H = H;
    a.W = W;
    a.P = particles_per_cell;
    a.S = step_limit;
    a.run = run_id;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);

    hipError_t e;
    // private rasters (counts then v^2 bits, contiguous), the internal stats and the per-XCD queues
    if ((e = avl::launch_fill_u32(ws.priv_counts, 0u, (int64_t)(ws.priv_vmax2 - ws.priv_counts) + avl::kXcds * n, s)) !=
        hipSuccess)
        return hip_fail(e, "avl_trajectories: zero rasters");
    if ((e = avl::launch_fill_u64(ws.stats, 0ull, 4 + 2 + avl::kXcds, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories: zero queues");
    if (stats && (e = avl::launch_fill_u64(a.stats, 0ull, 4, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories: zero stats");
    if ((e = avl::launch_compact(mask, n, ws.cells, ws.n_cells, ws.blk, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories: compaction");
    static thread_local int cached_dev = -1;
    static thread_local avl::LaunchShape cached_shape{256, 2048};
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "avl_trajectories: hipGetDevice");
    if (dev != cached_dev) {
        cached_shape = avl::trajectory_shape();
        cached_dev = dev;
    }
    if ((e = avl::launch_trajectories(a, cached_shape, s)) != hipSuccess) return hip_fail(e, "avl_trajectories: launch");
    if ((e = avl::launch_merge_rasters(ws.priv_counts, ws.priv_vmax2, n, counts, vmax, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories: merge");
    return AVL_OK;
}

}  // extern "C"
