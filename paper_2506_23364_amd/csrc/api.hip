// extern "C" entry points of libavl.so: host-side argument checks, workspace carving, kernel
// enqueueing, the autotuner of the trajectory kernel and the graph cache of batched calls.
// See include/avl.h for the contract of each call.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "avl_internal.h"

// Scratch of avl_trajectories_noalloc: the single-run workspace in a file-scope device array, one copy per
// GPU, which the code object's loader places in device memory and which lives until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host it only names the symbol): the device
// address comes from hipGetSymbolAddress, taken once per device with that device current.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace avl {

size_t workspace_bytes(int64_t H, int64_t W, int64_t mult) {
    const int64_t n = H * W * mult * mult;  // texels of the release texture
    return kControl + round256((size_t)scan_blocks(n) * sizeof(uint32_t)) + round256((size_t)n * sizeof(int32_t)) +
           round256((size_t)n * sizeof(StartRec)) +
           round256((size_t)padded_cells(H, W) * sizeof(float));
}

Workspace carve(void* base, int64_t H, int64_t W, int64_t mult) {
    const int64_t n = H * W * mult * mult;
    char* p = static_cast<char*>(base);
    Workspace w{};
    w.n_cells = reinterpret_cast<int32_t*>(p);
    w.stats = reinterpret_cast<unsigned long long*>(p + 64);
    w.queues = reinterpret_cast<unsigned long long*>(p + 512);
    w.run_off = reinterpret_cast<unsigned long long*>(p + 192);
    w.runs = reinterpret_cast<RunConst*>(p + 256);
    p += kControl;
    w.blk = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)scan_blocks(n) * sizeof(uint32_t));
    w.cells = reinterpret_cast<int32_t*>(p);
    p += round256((size_t)n * sizeof(int32_t));
    w.starts = reinterpret_cast<StartRec*>(p);
    p += round256((size_t)n * sizeof(StartRec));
    w.dem_pad = reinterpret_cast<float*>(p);
    return w;
}

size_t batched_workspace_bytes(int64_t H, int64_t W, int64_t n_tiles, int64_t n_masks, int64_t n_runs) {
    const int64_t n = H * W;
    return kControl + round256((size_t)scan_blocks(n) * sizeof(uint32_t)) +
           round256((size_t)n_masks * n * sizeof(int32_t)) + round256((size_t)n_masks * sizeof(int32_t)) +
           round256((size_t)n_runs * sizeof(RunConst)) + round256((size_t)(n_runs + 1) * sizeof(unsigned long long)) +
           round256((size_t)n_runs * 4 * sizeof(unsigned long long)) + round256((size_t)n_masks * sizeof(int32_t)) +
           round256((size_t)n_masks * n * sizeof(StartRec)) +
           round256((size_t)n_tiles * padded_cells(H, W) * sizeof(float));
}

Workspace carve_batched(void* base, int64_t H, int64_t W, int64_t n_masks, int64_t n_runs) {
    const int64_t n = H * W;
    char* p = static_cast<char*>(base);
    Workspace w{};
    w.queues = reinterpret_cast<unsigned long long*>(p + 512);
    p += kControl;
    w.blk = reinterpret_cast<uint32_t*>(p);
    p += round256((size_t)scan_blocks(n) * sizeof(uint32_t));
    w.cells = reinterpret_cast<int32_t*>(p);
    p += round256((size_t)n_masks * n * sizeof(int32_t));
    w.n_cells = reinterpret_cast<int32_t*>(p);
    p += round256((size_t)n_masks * sizeof(int32_t));
    w.runs = reinterpret_cast<RunConst*>(p);
    p += round256((size_t)n_runs * sizeof(RunConst));
    w.run_off = reinterpret_cast<unsigned long long*>(p);
    p += round256((size_t)(n_runs + 1) * sizeof(unsigned long long));
    w.stats = reinterpret_cast<unsigned long long*>(p);
    p += round256((size_t)n_runs * 4 * sizeof(unsigned long long));
    w.rec_run = reinterpret_cast<int32_t*>(p);
    p += round256((size_t)n_masks * sizeof(int32_t));
    w.starts = reinterpret_cast<StartRec*>(p);
    p += round256((size_t)n_masks * n * sizeof(StartRec));
    w.dem_pad = reinterpret_cast<float*>(p);
    return w;
}

// Smooth pass workspace: the single-run control block, scan sums and cell list, then the end records,
// checkpoints, per-particle adjoint results, reduction partials and the adjoint's scratch, the padded DEM,
// and per release cell its start state and the mass of each of its particles (made by the forward, read
// by the adjoint).
struct SmoothWs {
    Workspace w;
    StartRec* starts;
    float* mpc;
    uint32_t* end_rec;
    float* ck;
    float* pp;
    double* part;
    float2* scratch;
    float* dem_pad;
};

static size_t smooth_layout(int64_t H, int64_t W, int64_t cap_cells, uint32_t P, uint32_t S, char* base,
                            SmoothWs* out) {
    const int64_t n = H * W;
    const unsigned long long cap = (unsigned long long)cap_cells * P;
    const size_t C = smooth_checkpoints(S);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += round256(bytes);
        return at;
    };
    const size_t o_ctrl = take(kControl);
    const size_t o_blk = take((size_t)scan_blocks(n) * sizeof(uint32_t));
    const size_t o_cells = take((size_t)n * sizeof(int32_t));
    const size_t o_end = take((size_t)cap * sizeof(uint32_t));
    const size_t o_ck = take(5 * C * (size_t)cap * sizeof(float));
    const size_t o_pp = take(4 * (size_t)cap * sizeof(float));
    const size_t o_part = take(3 * smooth_reduce_blocks(cap) * sizeof(double));
    const size_t o_scr = take(smooth_scratch_bytes());
    const size_t o_pad = take((size_t)padded_cells(H, W) * sizeof(float));
    const size_t o_st = take((size_t)cap_cells * sizeof(StartRec));
    const size_t o_mpc = take((size_t)cap_cells * sizeof(float));
    if (base && out) {
        char* p = base + o_ctrl;
        out->w = Workspace{};
        out->starts = reinterpret_cast<StartRec*>(base + o_st);
        out->mpc = reinterpret_cast<float*>(base + o_mpc);
        out->w.n_cells = reinterpret_cast<int32_t*>(p);
        out->w.stats = reinterpret_cast<unsigned long long*>(p + 64);
        out->w.queues = reinterpret_cast<unsigned long long*>(p + 512);
        out->w.run_off = reinterpret_cast<unsigned long long*>(p + 192);
        out->w.runs = reinterpret_cast<RunConst*>(p + 256);
        out->w.blk = reinterpret_cast<uint32_t*>(base + o_blk);
        out->w.cells = reinterpret_cast<int32_t*>(base + o_cells);
        out->end_rec = reinterpret_cast<uint32_t*>(base + o_end);
        out->ck = reinterpret_cast<float*>(base + o_ck);
        out->pp = reinterpret_cast<float*>(base + o_pp);
        out->part = reinterpret_cast<double*>(base + o_part);
        out->scratch = reinterpret_cast<float2*>(base + o_scr);
        out->dem_pad = reinterpret_cast<float*>(base + o_pad);
    }
    return off;
}

}  // namespace avl

namespace {

thread_local std::string g_last_error;
thread_local int32_t g_last_variant = -1;

// kernel timing (avl_set_profiling): events around the last uncaptured trajectory launch
bool g_profile = false;
// tail probe (avl_set_probe): device buffer of 3 u64 per block of the trajectory grid, or null
unsigned long long* g_probe = nullptr;
uint64_t g_probe_blocks = 0;
bool g_profile_valid = false;
hipEvent_t g_prof_ev[2] = {nullptr, nullptr};

bool capturing(hipStream_t s);

// Enqueues `launch` (one kernel), bracketed by the timing events when profiling is on and the stream is
// not being captured.
template <class Launch>
hipError_t timed(hipStream_t s, Launch launch) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool on = g_profile && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
    hipError_t e;
    if (on && (e = hipEventRecord(g_prof_ev[0], s)) != hipSuccess) return e;
    if ((e = launch()) != hipSuccess) return e;
    if (on) {
        if ((e = hipEventRecord(g_prof_ev[1], s)) != hipSuccess) return e;
        g_profile_valid = true;
    }
    return hipSuccess;
}

// The trajectory kernel, timed as above; an uncaptured single run also writes the tail probe when one is set
// and holds the grid.
hipError_t timed_launch(const avl::TrajArgs& a, bool batched, const avl::LaunchShape& sh, hipStream_t s) {
    avl::TrajArgs b = a;
    if (!batched && g_probe && (uint64_t)sh.grid <= g_probe_blocks && !capturing(s)) b.probe = g_probe;
    return timed(s, [&] { return avl::launch_trajectories(b, batched, sh, s); });
}

__attribute__((format(printf, 2, 3))) int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
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

// ------------------------------------------------------------------ tuning state
std::mutex g_mu;
int32_t g_variant_override = -1;
int32_t g_smooth_override[2] = {-1, -1};  // smooth forward, adjoint
bool g_graphs = true;
std::map<std::vector<int64_t>, int> g_best;  // (device, batched, size buckets) -> variant

int ilog2(uint64_t v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

std::vector<int64_t> tune_key(bool batched, int64_t n, int64_t n_runs, uint32_t P, uint32_t S) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return {dev, batched ? 1 : 0, ilog2((uint64_t)n), ilog2((uint64_t)n_runs), ilog2(P), ilog2((uint64_t)S + 1)};
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Variant for this problem: the override, the cached choice, or (first time, not under capture) the
// fastest of all variants, each timed once with HIP events after `zero` re-zeroes what the kernel
// accumulates into. The inputs of the kernel (cell lists, run table) must already be enqueued.
// may_tune = false: never time the variants here (the allocation-free entry point creates no events); an
// uncached problem then takes variant 0.
template <class Zero>
hipError_t choose_variant(const avl::TrajArgs& a, bool batched, const std::vector<int64_t>& key, hipStream_t s,
                          Zero zero, int* variant, bool may_tune = true) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_variant_override >= 0) {
            *variant = g_variant_override;
            return hipSuccess;
        }
        auto it = g_best.find(key);
        if (it != g_best.end()) {
            *variant = it->second;
            return hipSuccess;
        }
    }
    if (!may_tune || capturing(s)) {
        *variant = 0;
        return hipSuccess;
    }
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    // Each variant's time is the minimum over kTuneRounds launches, the rounds interleaved: the first
    // launch of a kernel also pays for loading its code, and the variants differ by a few percent.
    constexpr int kTuneRounds = 5;
    const int nv = avl::trajectory_variants();
    std::vector<float> vmin(nv, 1e30f);
    e = hipSuccess;
    for (int round = 0; round < kTuneRounds && e == hipSuccess; ++round) {
        for (int v = 0; v < nv; ++v) {
            const avl::LaunchShape sh = avl::trajectory_shape(batched, v);
            if ((e = zero()) != hipSuccess) break;
            if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
            if ((e = avl::launch_trajectories(a, batched, sh, s)) != hipSuccess) break;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (ms < vmin[v]) vmin[v] = ms;
        }
    }
    // a later variant replaces the current choice only when it is at least kTuneMargin faster: closer
    // timings are within the run-to-run spread, and variant 0 is the one measured best on the workloads
    constexpr float kTuneMargin = 0.98f;
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (vmin[v] < vmin[best] * kTuneMargin) best = v;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    g_best[key] = best;
    *variant = best;
    return hipSuccess;
}

// The same for the smooth kernels' grid variants: `launch(v)` enqueues variant v after `zero()` re-zeroes what
// it accumulates into; the fastest of kTuneRounds interleaved timings is kept per key (kind 2: forward, 3:
// adjoint). Under capture, or with may_tune false, an uncached key takes variant 0.
template <class Zero, class Launch>
hipError_t choose_smooth(const std::vector<int64_t>& key, int nv, hipStream_t s, Zero zero, Launch launch, int* variant,
                         bool may_tune = true) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const int32_t forced = g_smooth_override[key[1] == 2 ? 0 : 1];
        if (forced >= 0) {
            *variant = forced < nv ? forced : 0;
            return hipSuccess;
        }
        auto it = g_best.find(key);
        if (it != g_best.end()) {
            *variant = it->second;
            return hipSuccess;
        }
    }
    if (!may_tune || capturing(s) || nv <= 1) {
        *variant = 0;
        return hipSuccess;
    }
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    constexpr int kTuneRounds = 3;
    std::vector<float> vmin(nv, 1e30f);
    for (int round = 0; round < kTuneRounds && e == hipSuccess; ++round) {
        for (int v = 0; v < nv; ++v) {
            if ((e = zero()) != hipSuccess) break;
            if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
            if ((e = launch(v)) != hipSuccess) break;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (ms < vmin[v]) vmin[v] = ms;
        }
    }
    constexpr float kTuneMargin = 0.98f;
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (vmin[v] < vmin[best] * kTuneMargin) best = v;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    g_best[key] = best;
    *variant = best;
    return hipSuccess;
}

std::vector<int64_t> smooth_key(int kind, int64_t n, int64_t cap, uint32_t P, uint32_t S) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return {dev, kind, ilog2((uint64_t)n), ilog2((uint64_t)cap + 1), ilog2(P), ilog2((uint64_t)S + 1)};
}

// ------------------------------------------------------------------ graph cache of batched calls
struct GraphEntry {
    hipGraphExec_t exec;
    uint64_t last_use;
};
std::map<std::vector<uint64_t>, GraphEntry> g_graph_cache;
uint64_t g_clock = 0;
constexpr size_t kMaxGraphs = 16;

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

int avl_set_tuning(int32_t variant, int32_t graphs) {
    if (variant < -1 || variant >= avl::trajectory_variants()) return AVL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_variant_override = variant;
    g_graphs = graphs != 0;
    return AVL_OK;
}

int32_t avl_tuning_variants(void) { return avl::trajectory_variants(); }

int avl_set_smooth_tuning(int32_t forward_variant, int32_t backward_variant) {
    if (forward_variant < -1 || forward_variant >= avl::smooth_forward_variants() || backward_variant < -1 ||
        backward_variant >= avl::smooth_backward_variants())
        return AVL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_smooth_override[0] = forward_variant;
    g_smooth_override[1] = backward_variant;
    return AVL_OK;
}

int avl_smooth_tuning_variants(int32_t* n_forward, int32_t* n_backward) {
    g_last_error.clear();
    if (!n_forward || !n_backward) return fail(AVL_EINVAL, "avl_smooth_tuning_variants: null pointer");
    *n_forward = avl::smooth_forward_variants();
    *n_backward = avl::smooth_backward_variants();
    return AVL_OK;
}

int avl_tuning_variant_info(int32_t variant, int32_t* info) {
    g_last_error.clear();
    if (!info) return fail(AVL_EINVAL, "avl_tuning_variant_info: info is NULL");
    if (!avl::trajectory_variant_info(variant, info))
        return fail(AVL_EINVAL, "avl_tuning_variant_info: variant out of range");
    return AVL_OK;
}

int32_t avl_mipmap_levels(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    int32_t n = 1;
    for (int32_t m = H > W ? H : W; m > 1; m = (m + 1) / 2) ++n;
    return n;
}

int64_t avl_mipmap_cells(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    int64_t total = 0, h = H, w = W;
    while (h > 1 || w > 1) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
        total += h * w;
    }
    return total;
}

int avl_overlay_mipmap(const uint32_t* counts, const float* vmax, int32_t H, int32_t W, uint64_t* counts_pyr,
                       float* vmax_pyr, void* stream) {
    g_last_error.clear();
    if (!counts || !vmax || !counts_pyr || !vmax_pyr) return fail(AVL_EINVAL, "avl_overlay_mipmap: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_overlay_mipmap: need H, W >= 1 and H*W < 2^31");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t L = avl_mipmap_levels(H, W);
    const void* cin = counts;
    bool cin64 = false;
    const float* vin = vmax;
    int h0 = H, w0 = W, done = 1;
    int64_t at = 0;
    auto* cp = reinterpret_cast<unsigned long long*>(counts_pyr);
    while (done < L) {
        avl::MipLevels o{};
        const int nlev = (L - done) < avl::kMipPass ? (L - done) : avl::kMipPass;
        int h = h0, w = w0;
        for (int l = 0; l < nlev; ++l) {
            h = (h + 1) / 2;
            w = (w + 1) / 2;
            o.c[l] = cp + at;
            o.v[l] = vmax_pyr + at;
            o.h[l] = h;
            o.w[l] = w;
            at += (int64_t)h * w;
        }
        hipError_t e;
        if ((e = avl::launch_mip_pass(cin, cin64, vin, h0, w0, nlev, o, s)) != hipSuccess)
            return hip_fail(e, "avl_overlay_mipmap");
        cin = o.c[nlev - 1];
        cin64 = true;
        vin = o.v[nlev - 1];
        h0 = o.h[nlev - 1];
        w0 = o.w[nlev - 1];
        done += nlev;
    }
    return AVL_OK;
}

int32_t avl_last_variant(void) { return g_last_variant; }

int avl_set_profiling(int32_t enable) {
    g_last_error.clear();
    if (enable && !g_prof_ev[0]) {
        hipError_t e;
        if ((e = hipEventCreate(&g_prof_ev[0])) != hipSuccess) return hip_fail(e, "avl_set_profiling");
        if ((e = hipEventCreate(&g_prof_ev[1])) != hipSuccess) return hip_fail(e, "avl_set_profiling");
    }
    g_profile = enable != 0;
    g_profile_valid = false;
    return AVL_OK;
}

int avl_set_probe(uint64_t* blocks3, uint64_t n_blocks) {
    g_last_error.clear();
    g_probe = reinterpret_cast<unsigned long long*>(blocks3);
    g_probe_blocks = blocks3 ? n_blocks : 0;
    return AVL_OK;
}

int32_t avl_trajectory_grid(int32_t variant) {
    if (variant < 0 || variant >= avl::trajectory_variants()) return -1;
    return avl::trajectory_shape(false, variant).grid;
}

int avl_last_kernel_ms(float* ms) {
    g_last_error.clear();
    if (!ms) return fail(AVL_EINVAL, "avl_last_kernel_ms: null pointer");
    if (!g_profile_valid) return fail(AVL_EINVAL, "avl_last_kernel_ms: no timed trajectory call");
    hipError_t e;
    if ((e = hipEventSynchronize(g_prof_ev[1])) != hipSuccess) return hip_fail(e, "avl_last_kernel_ms");
    if ((e = hipEventElapsedTime(ms, g_prof_ev[0], g_prof_ev[1])) != hipSuccess)
        return hip_fail(e, "avl_last_kernel_ms");
    return AVL_OK;
}

size_t avl_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    return avl::workspace_bytes(H, W);
}

size_t avl_batched_workspace_bytes(int32_t H, int32_t W, int32_t n_tiles, int32_t n_masks, int32_t n_runs) {
    if (H < 1 || W < 1 || n_tiles < 1 || n_masks < 1 || n_runs < 1) return 0;
    return avl::batched_workspace_bytes(H, W, n_tiles, n_masks, n_runs);
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

namespace {
// checks of the release criteria; the cosines of the slope range, taken in binary64 and rounded once
const char* release_bounds(float slope_min_deg, float slope_max_deg, float z_min, float z_max, float* cmin,
                           float* cmax) {
    if (!(slope_min_deg >= 0.0f && slope_min_deg <= slope_max_deg && slope_max_deg <= 90.0f))
        return "need 0 <= slope_min_deg <= slope_max_deg <= 90";
    if (std::isnan(z_min) || std::isnan(z_max)) return "NaN elevation bound";
    const double d2r = 3.14159265358979323846 / 180.0;
    *cmin = (float)std::cos((double)slope_max_deg * d2r);
    *cmax = (float)std::cos((double)slope_min_deg * d2r);
    return nullptr;
}
}  // namespace

int avl_normals_release_mask(const float* dem, int32_t H, int32_t W, float cell_size, float slope_min_deg,
                             float slope_max_deg, float z_min, float z_max, float* normals4, uint8_t* mask,
                             void* stream) {
    g_last_error.clear();
    if (!dem || !normals4 || !mask) return fail(AVL_EINVAL, "avl_normals_release_mask: null pointer");
    if (!grid_ok(H, W, 2)) return fail(AVL_EINVAL, "avl_normals_release_mask: need H, W >= 2 and H*W < 2^31");
    if (!finite(cell_size) || !(cell_size > 0.0f))
        return fail(AVL_EINVAL, "avl_normals_release_mask: cell_size must be > 0");
    if (reinterpret_cast<uintptr_t>(normals4) & 15)
        return fail(AVL_EINVAL, "avl_normals_release_mask: normals4 not 16-byte aligned");
    float cmin, cmax;
    if (const char* why = release_bounds(slope_min_deg, slope_max_deg, z_min, z_max, &cmin, &cmax))
        return fail(AVL_EINVAL, "avl_normals_release_mask: %s", why);
    hipError_t e = avl::launch_normals_mask(dem, H, W, cell_size, cmin, cmax, z_min, z_max, normals4, mask,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_normals_release_mask");
}

int avl_release_mask(const float* normals4, const float* dem, int32_t H, int32_t W, float slope_min_deg,
                     float slope_max_deg, float z_min, float z_max, uint8_t* mask, void* stream) {
    g_last_error.clear();
    if (!normals4 || !dem || !mask) return fail(AVL_EINVAL, "avl_release_mask: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_release_mask: need H, W >= 1 and H*W < 2^31");
    if (reinterpret_cast<uintptr_t>(normals4) & 15)
        return fail(AVL_EINVAL, "avl_release_mask: normals4 not 16-byte aligned");
    float cmin, cmax;
    if (const char* why = release_bounds(slope_min_deg, slope_max_deg, z_min, z_max, &cmin, &cmax))
        return fail(AVL_EINVAL, "avl_release_mask: %s", why);
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
    if (workspace_bytes < avl::workspace_bytes(H, W)) return fail(AVL_ENOMEM, "avl_release_cells: workspace too small");
    avl::Workspace ws = avl::carve(workspace, H, W);
    hipError_t e = avl::launch_compact(mask, n, cells, n_cells, ws.blk, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_release_cells");
}

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of that device's copy of `scratch`

hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return hipSuccess;
}

// Path recording of a pass (avl_trajectories_record).
struct Record {
    uint64_t first;
    uint32_t n, stride;
    const uint64_t* offsets;
    float* points;
    float* speeds2;
    uint32_t* ends;
};

// One trajectory pass from a release texture with mult x mult texels per DEM cell (mask: mult*H x mult*W).
// noalloc: ignore workspace / workspace_bytes and run in the current device's `scratch` (no allocation,
// no event creation, no tuning). rec: run the recording instantiation instead of the tuned variants.
int single_pass(const char* where, const float* dem, const uint8_t* mask, int32_t H, int32_t W, int32_t mult,
                float cell_size, const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit,
                uint64_t seed, uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                size_t workspace_bytes, void* stream, bool noalloc = false, const Record* rec = nullptr) {
    if (!dem || !mask || !counts || !vmax || (!noalloc && !workspace))
        return fail(AVL_EINVAL, "%s: null pointer", where);
    if (!grid_ok(H, W, 1) || avl::padded_cells(H, W) >= (int64_t(1) << 30))
        return fail(AVL_EINVAL, "%s: need H, W >= 1 and (H + 2)(W + 2) < 2^30", where);
    if (mult < 1 || mult > AVL_MAX_RELEASE_MULT)
        return fail(AVL_EINVAL, "%s: release texels per DEM cell edge must be in [1, %d]", where, AVL_MAX_RELEASE_MULT);
    if ((int64_t)H * W * mult * mult >= (int64_t(1) << 31))
        return fail(AVL_EINVAL, "%s: need (mult H)(mult W) < 2^31", where);
    // release points (k + 1/2) / mult are formed in binary32: below 2^23 texels per row and column the
    // numerator is exact and the quotient's rounding error stays under the 1/(2 mult) margin to the next
    // cell edge, so the DEM cell under each release point is the exact one
    if ((int64_t)mult * W >= (int64_t(1) << 23) || (int64_t)mult * H >= (int64_t(1) << 23))
        return fail(AVL_EINVAL, "%s: need mult W and mult H < 2^23", where);
    if (!finite(cell_size) || !(cell_size > 0.0f)) return fail(AVL_EINVAL, "%s: cell_size must be > 0", where);
    if (particles_per_cell == 0) return fail(AVL_EINVAL, "%s: particles_per_cell must be >= 1", where);
    if (const char* why = check_params(params)) return fail(AVL_EINVAL, "%s: %s", where, why);
    const int64_t n = (int64_t)H * W;
    const int64_t nf = n * mult * mult;
    if (noalloc) {
        const size_t need = avl::workspace_bytes(H, W, mult);
        if (need > kScratchBytes)
            return fail(AVL_EINVAL, "%s: the grid needs %zu bytes of scratch, more than the %zu bytes it holds", where,
                        need, kScratchBytes);
        hipError_t e = scratch_address(&workspace);
        if (e != hipSuccess) return hip_fail(e, (std::string(where) + ": scratch address").c_str());
        workspace_bytes = kScratchBytes;
    }
    if (workspace_bytes < avl::workspace_bytes(H, W, mult)) return fail(AVL_ENOMEM, "%s: workspace too small", where);
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::Workspace ws = avl::carve(workspace, H, W, mult);

    avl::TrajArgs a{};
    a.dem = dem;
    a.cells = ws.cells;
    a.runs = ws.runs;
    a.run_off = ws.run_off;
    a.queues = ws.queues;
    a.counts = counts;
    a.vmax2 = reinterpret_cast<uint32_t*>(vmax);  // v^2 bits during the kernel, speeds after the finalize
    a.stats = stats ? reinterpret_cast<unsigned long long*>(stats) : ws.stats;
    a.H = H;
    a.W = W;
    a.n_runs = 1;
    a.S = step_limit;
    a.g2 = 9.81f + 9.81f;
    a.starts = ws.starts;
    a.pdiv = avl::make_divu32(particles_per_cell);
    a.dem_pad = ws.dem_pad;
    a.pad_bytes = (uint32_t)(avl::padded_cells(H, W) * sizeof(float));
    a.runout_angle = params->tan_alpha >= 0.0f ? 1u : 0u;
    a.wdiv = avl::make_divu32((uint32_t)W);

    auto zero = [&]() -> hipError_t {
        hipError_t e;
        if ((e = avl::launch_fill_u32(counts, 0u, n, s)) != hipSuccess) return e;
        if ((e = avl::launch_fill_u32(a.vmax2, 0u, n, s)) != hipSuccess) return e;
        if ((e = avl::launch_fill_u64(ws.queues, 0ull, avl::kXcds * avl::kQueueStride, s)) != hipSuccess) return e;
        return avl::launch_fill_u64(a.stats, 0ull, 4, s);
    };
    hipError_t e;
    if ((e = avl::launch_compact(mask, nf, ws.cells, ws.n_cells, ws.blk, s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": compaction").c_str());
    if ((e = avl::launch_start_records(dem, H, W, mult, ws.cells, ws.n_cells, nf, ws.starts, s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": start records").c_str());
    if ((e = avl::launch_pad_dem(dem, H, W, ws.dem_pad, s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": padded DEM").c_str());
    const avl::RunSpec spec{0u, 0u, 0u, run_id, (unsigned long long)seed};
    if ((e = avl::launch_setup_runs(nullptr, nullptr, 0, spec, *params, ws.n_cells, 1, 1, 1, H, W, cell_size,
                                    particles_per_cell, false, ws.runs, ws.run_off, nullptr, s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": run setup").c_str());
    if (rec) {
        a.rec_first = rec->first;
        a.rec_n = rec->n;
        a.rec_stride = rec->stride;
        a.rec_off = reinterpret_cast<const unsigned long long*>(rec->offsets);
        a.rec_xy = reinterpret_cast<float2*>(rec->points);
        a.rec_v2 = rec->speeds2;
        a.rec_end = rec->ends;
        if ((e = zero()) != hipSuccess || (e = avl::launch_fill_u32(rec->ends, ~0u, rec->n, s)) != hipSuccess)
            return hip_fail(e, (std::string(where) + ": zero").c_str());
        if ((e = timed(s, [&] { return avl::launch_trajectories_record(a, s); })) != hipSuccess)
            return hip_fail(e, (std::string(where) + ": launch").c_str());
        if ((e = avl::launch_finalize_vmax(a.vmax2, n, s)) != hipSuccess)
            return hip_fail(e, (std::string(where) + ": finalize").c_str());
        return AVL_OK;
    }
    int variant = 0;
    if ((e = choose_variant(a, false, tune_key(false, nf, 1, particles_per_cell, step_limit), s, zero, &variant,
                            !noalloc)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": autotune").c_str());
    g_last_variant = variant;
    if ((e = zero()) != hipSuccess) return hip_fail(e, (std::string(where) + ": zero").c_str());
    if ((e = timed_launch(a, false, avl::trajectory_shape(false, variant), s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": launch").c_str());
    if ((e = avl::launch_finalize_vmax(a.vmax2, n, s)) != hipSuccess)
        return hip_fail(e, (std::string(where) + ": finalize").c_str());
    return AVL_OK;
}

}  // namespace

int avl_trajectories(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                     const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                     uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                     size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    return single_pass("avl_trajectories", dem, mask, H, W, 1, cell_size, params, particles_per_cell, step_limit,
                       seed, run_id, counts, vmax, stats, workspace, workspace_bytes, stream);
}

int avl_trajectories_noalloc(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                             const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit,
                             uint64_t seed, uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats,
                             void* stream) {
    g_last_error.clear();
    return single_pass("avl_trajectories_noalloc", dem, mask, H, W, 1, cell_size, params, particles_per_cell,
                       step_limit, seed, run_id, counts, vmax, stats, nullptr, 0, stream, true);
}

size_t avl_noalloc_scratch_bytes(void) { return kScratchBytes; }

int avl_trajectories_record(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                            const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                            uint32_t run_id, uint64_t first, uint32_t n_rec, const uint64_t* offsets, uint32_t stride,
                            float* points, float* speeds2, uint32_t* ends, uint32_t* counts, float* vmax,
                            uint64_t* stats, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (n_rec == 0 || !ends) return fail(AVL_EINVAL, "avl_trajectories_record: need n_rec >= 1 and ends");
    if (first > ~0ull - n_rec) return fail(AVL_EINVAL, "avl_trajectories_record: first + n_rec overflows");
    if (speeds2 && !points) return fail(AVL_EINVAL, "avl_trajectories_record: speeds2 needs points");
    if (points && !offsets && stride == 0)
        return fail(AVL_EINVAL, "avl_trajectories_record: points need offsets or a stride >= 1");
    if (points && !offsets && (uint64_t)n_rec * stride >= (uint64_t(1) << 40))
        return fail(AVL_EINVAL, "avl_trajectories_record: n_rec * stride must be < 2^40");
    const Record rec{first, n_rec, stride, offsets, points, speeds2, ends};
    return single_pass("avl_trajectories_record", dem, mask, H, W, 1, cell_size, params, particles_per_cell,
                       step_limit, seed, run_id, counts, vmax, stats, workspace, workspace_bytes, stream, false, &rec);
}

int avl_bench_schedule(int32_t mode, int32_t H, int32_t W, const float* points, const float* speeds2,
                       const uint64_t* offsets, const uint32_t* ends, uint64_t n_particles, uint64_t* totals,
                       const uint64_t* gather_base, const uint64_t* visit_base, uint32_t* gathers, uint32_t* visits,
                       void* stream) {
    g_last_error.clear();
    if (mode != 0 && mode != 1) return fail(AVL_EINVAL, "avl_bench_schedule: mode must be 0 or 1");
    if (!points || !speeds2 || !offsets || !ends) return fail(AVL_EINVAL, "avl_bench_schedule: null pointer");
    if (mode == 0 && !totals) return fail(AVL_EINVAL, "avl_bench_schedule: totals is NULL");
    if (mode == 1 && (!gather_base || !visit_base || !gathers || !visits))
        return fail(AVL_EINVAL, "avl_bench_schedule: null pointer");
    if (!grid_ok(H, W, 1) || H >= (1 << 23) || W >= (1 << 23) || avl::padded_cells(H, W) >= (int64_t(1) << 30))
        return fail(AVL_EINVAL, "avl_bench_schedule: need H, W >= 1, H, W < 2^23 and (H + 2)(W + 2) < 2^30");
    if (n_particles == 0) return AVL_OK;
    hipError_t e = avl::launch_replay_schedule(
        mode, reinterpret_cast<const float2*>(points), speeds2, reinterpret_cast<const unsigned long long*>(offsets),
        ends, n_particles, W, reinterpret_cast<unsigned long long*>(totals),
        reinterpret_cast<const unsigned long long*>(gather_base), reinterpret_cast<const unsigned long long*>(visit_base),
        gathers, reinterpret_cast<uint2*>(visits), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_bench_schedule");
}

int avl_bench_gather(const float* dem, int32_t H, int32_t W, const uint32_t* gathers, uint64_t n_gathers,
                     uint32_t* checksum, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    if (!dem || !gathers || !checksum || !workspace) return fail(AVL_EINVAL, "avl_bench_gather: null pointer");
    if (!grid_ok(H, W, 1) || avl::padded_cells(H, W) >= (int64_t(1) << 30) || H >= (1 << 23) || W >= (1 << 23))
        return fail(AVL_EINVAL, "avl_bench_gather: need H, W >= 1, H, W < 2^23 and (H + 2)(W + 2) < 2^30");
    if (workspace_bytes < avl::workspace_bytes(H, W)) return fail(AVL_ENOMEM, "avl_bench_gather: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::Workspace ws = avl::carve(workspace, H, W);
    hipError_t e;
    if ((e = avl::launch_pad_dem(dem, H, W, ws.dem_pad, s)) != hipSuccess ||
        (e = avl::launch_fill_u32(checksum, 0u, 1, s)) != hipSuccess)
        return hip_fail(e, "avl_bench_gather: set-up");
    if (n_gathers == 0) return AVL_OK;
    const uint32_t pad_bytes = (uint32_t)(avl::padded_cells(H, W) * sizeof(float));
    e = timed(s, [&] {
        return avl::launch_replay_gather(gathers, n_gathers, ws.dem_pad, pad_bytes, 4u * ((uint32_t)W + 2u), checksum,
                                         s);
    });
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_bench_gather: launch");
}

int avl_bench_atomics(int32_t H, int32_t W, const uint32_t* visits, uint64_t n_visits, uint32_t* counts,
                      uint32_t* vmax2_bits, void* stream) {
    g_last_error.clear();
    if (!visits || !counts || !vmax2_bits) return fail(AVL_EINVAL, "avl_bench_atomics: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_bench_atomics: need H, W >= 1 and H*W < 2^31");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = (int64_t)H * W;
    hipError_t e;
    if ((e = avl::launch_fill_u32(counts, 0u, n, s)) != hipSuccess ||
        (e = avl::launch_fill_u32(vmax2_bits, 0u, n, s)) != hipSuccess)
        return hip_fail(e, "avl_bench_atomics: set-up");
    if (n_visits == 0) return AVL_OK;
    e = timed(s, [&] {
        return avl::launch_replay_atomics(reinterpret_cast<const uint2*>(visits), n_visits, counts, vmax2_bits, s);
    });
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_bench_atomics: launch");
}

int avl_bench_stream(const void* src, void* dst, size_t bytes, void* stream) {
    g_last_error.clear();
    if (!src || !dst) return fail(AVL_EINVAL, "avl_bench_stream: null pointer");
    if (bytes % 16 || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
        return fail(AVL_EINVAL, "avl_bench_stream: bytes and both pointers must be multiples of 16");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(s, [&] { return avl::launch_stream_copy(src, dst, bytes / 16, s); });
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_bench_stream");
}

int avl_snow_cover(const float* normals4, const float* dem, int32_t H, int32_t W, float snow_line, float alt_blend,
                   float max_slope_deg, float slope_blend_deg, float* alpha, void* stream) {
    g_last_error.clear();
    if (!normals4 || !dem || !alpha) return fail(AVL_EINVAL, "avl_snow_cover: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_snow_cover: need H, W >= 1 and H*W < 2^31");
    if (reinterpret_cast<uintptr_t>(normals4) & 15)
        return fail(AVL_EINVAL, "avl_snow_cover: normals4 not 16-byte aligned");
    if (!finite(snow_line) || !finite(alt_blend) || !(alt_blend >= 0.0f))
        return fail(AVL_EINVAL, "avl_snow_cover: need a finite snow line and a finite alt_blend >= 0");
    if (!(slope_blend_deg >= 0.0f && slope_blend_deg <= max_slope_deg && max_slope_deg <= 90.0f))
        return fail(AVL_EINVAL, "avl_snow_cover: need 0 <= slope_blend_deg <= max_slope_deg <= 90");
    const double d2r = 3.14159265358979323846 / 180.0;
    const float c_lo = (float)std::cos((double)max_slope_deg * d2r);
    const float c_hi = (float)std::cos(((double)max_slope_deg - (double)slope_blend_deg) * d2r);
    const float z_hi = snow_line + alt_blend;
    hipError_t e = avl::launch_snow_cover(normals4, dem, (int64_t)H * W, snow_line, z_hi, c_lo, c_hi, alpha,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_snow_cover");
}

size_t avl_fine_workspace_bytes(int32_t H, int32_t W, int32_t mult) {
    if (H < 1 || W < 1 || mult < 1 || mult > AVL_MAX_RELEASE_MULT) return 0;
    return avl::workspace_bytes(H, W, mult);
}

int avl_release_mask_fine(const float* normals4, const float* dem, int32_t H, int32_t W, int32_t mult,
                          float slope_min_deg, float slope_max_deg, float z_min, float z_max, uint8_t* mask,
                          void* stream) {
    g_last_error.clear();
    if (!normals4 || !dem || !mask) return fail(AVL_EINVAL, "avl_release_mask_fine: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_release_mask_fine: need H, W >= 1 and H*W < 2^31");
    if (mult < 1 || mult > AVL_MAX_RELEASE_MULT)
        return fail(AVL_EINVAL, "avl_release_mask_fine: mult must be in [1, %d]", AVL_MAX_RELEASE_MULT);
    if ((int64_t)H * W * mult * mult >= (int64_t(1) << 31))
        return fail(AVL_EINVAL, "avl_release_mask_fine: need (mult H)(mult W) < 2^31");
    if ((int64_t)mult * W >= (int64_t(1) << 23) || (int64_t)mult * H >= (int64_t(1) << 23))
        return fail(AVL_EINVAL, "avl_release_mask_fine: need mult W and mult H < 2^23");
    if (reinterpret_cast<uintptr_t>(normals4) & 15)
        return fail(AVL_EINVAL, "avl_release_mask_fine: normals4 not 16-byte aligned");
    if (!(slope_min_deg >= 0.0f && slope_min_deg <= slope_max_deg && slope_max_deg <= 90.0f))
        return fail(AVL_EINVAL, "avl_release_mask_fine: need 0 <= slope_min_deg <= slope_max_deg <= 90");
    if (std::isnan(z_min) || std::isnan(z_max)) return fail(AVL_EINVAL, "avl_release_mask_fine: NaN elevation bound");
    const double d2r = 3.14159265358979323846 / 180.0;
    const float cmin = (float)std::cos((double)slope_max_deg * d2r);
    const float cmax = (float)std::cos((double)slope_min_deg * d2r);
    hipError_t e = avl::launch_release_mask_fine(normals4, dem, H, W, mult, cmin, cmax, z_min, z_max, mask,
                                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_release_mask_fine");
}

int avl_trajectories_fine(const float* dem, const uint8_t* mask, int32_t H, int32_t W, int32_t mult, float cell_size,
                          const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                          uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                          size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    return single_pass("avl_trajectories_fine", dem, mask, H, W, mult, cell_size, params, particles_per_cell,
                       step_limit, seed, run_id, counts, vmax, stats, workspace, workspace_bytes, stream);
}

size_t avl_smooth_workspace_bytes(int32_t H, int32_t W, int32_t max_release_cells, uint32_t particles_per_cell,
                                  uint32_t step_limit) {
    if (H < 1 || W < 1 || max_release_cells < 0 || particles_per_cell == 0) return 0;
    return avl::smooth_layout(H, W, max_release_cells, particles_per_cell, step_limit, nullptr, nullptr);
}

namespace {

// shared argument checks of the smooth forward and the adjoint
int smooth_checks(const char* where, const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                  const avl_params* params, uint32_t P, uint32_t S, int32_t max_release_cells, void* workspace,
                  size_t workspace_bytes) {
    if (!dem || !mask || !workspace) return fail(AVL_EINVAL, "%s: null pointer", where);
    if (!grid_ok(H, W, 1) || avl::padded_cells(H, W) >= (int64_t(1) << 30))
        return fail(AVL_EINVAL, "%s: need H, W >= 1 and (H + 2)(W + 2) < 2^30", where);
    // the padded patch's row offset is a 24-bit product (W + 2 < 2^24), and positions are binary32
    if (H >= (1 << 23) || W >= (1 << 23)) return fail(AVL_EINVAL, "%s: need H, W < 2^23", where);
    if (!finite(cell_size) || !(cell_size > 0.0f)) return fail(AVL_EINVAL, "%s: cell_size must be > 0", where);
    if (P == 0) return fail(AVL_EINVAL, "%s: particles_per_cell must be >= 1", where);
    if (max_release_cells < 0 || (int64_t)max_release_cells > (int64_t)H * W)
        return fail(AVL_EINVAL, "%s: need 0 <= max_release_cells <= H*W", where);
    if ((uint64_t)max_release_cells * P >= (1ull << 32))
        return fail(AVL_EINVAL, "%s: max_release_cells * particles_per_cell must be < 2^32", where);
    if (S >= (1u << 30)) return fail(AVL_EINVAL, "%s: step_limit must be < 2^30", where);
    if (const char* why = check_params(params)) return fail(AVL_EINVAL, "smooth pass: %s", why);
    if (workspace_bytes < avl_smooth_workspace_bytes(H, W, max_release_cells, P, S))
        return fail(AVL_ENOMEM, "%s: workspace too small", where);
    return AVL_OK;
}

avl::SmoothArgs smooth_args(const float* dem, const float* mass, int32_t H, int32_t W, float cell_size,
                            const avl_params* params, uint32_t P, uint32_t S, int32_t max_release_cells,
                            const avl::SmoothWs& sw) {
    avl::SmoothArgs a{};
    a.dem = dem;
    a.mass = mass;
    a.cells = sw.w.cells;
    a.runs = sw.w.runs;
    a.run_off = sw.w.run_off;
    a.queues = sw.w.queues;
    a.ck = sw.ck;
    a.end_rec = sw.end_rec;
    a.pp = sw.pp;
    a.scratch = sw.scratch;
    a.H = H;
    a.W = W;
    a.S = S;
    a.C = (uint32_t)avl::smooth_checkpoints(S);
    a.cap = (unsigned long long)max_release_cells * P;
    const float g = 9.81f;
    a.g2 = g + g;
    const float dl = params->step_cells * cell_size;
    a.g2dl = a.g2 * dl;
    a.xi = params->xi;
    a.h = params->flow_height;
    a.dem_pad = sw.dem_pad;
    a.pad_bytes = (uint32_t)(avl::padded_cells(H, W) * sizeof(float));
    a.starts = sw.starts;
    a.mpc = sw.mpc;
    a.pdiv = avl::make_divu32(P);
    return a;
}

}  // namespace

namespace {
// The smooth forward pass. `prepared`: the workspace already holds this mask's release cells, padded DEM,
// start records and per-particle masses from an earlier pass with the same DEM, mask, mass and particles per
// cell (a calibration loop, where only the friction parameters change between passes), so only the run
// constants are set up again. `p_dev`, `spec_dev` (nullable, together): the run constants are set up from
// these device copies of the parameters and the run (a loop that updates the parameters on the device);
// `params` then serves only for the host checks of the parameters the loop does not change.
int smooth_forward(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                   float cell_size, const avl_params* params, uint32_t particles_per_cell,
                   uint32_t step_limit, uint64_t seed, uint32_t run_id, int32_t max_release_cells,
                   uint32_t flags, int64_t* deposit_q, float* deposit, int64_t* velocity_q, float* velocity,
                   uint64_t* stats, int32_t* status, void* workspace, size_t workspace_bytes, void* stream,
                   bool prepared, const avl_params* p_dev = nullptr, const avl::RunSpec* spec_dev = nullptr) {
    g_last_error.clear();
    int rc = smooth_checks("avl_trajectories_smooth", dem, mask, H, W, cell_size, params, particles_per_cell,
                           step_limit, max_release_cells, workspace, workspace_bytes);
    if (rc != AVL_OK) return rc;
    if (!deposit_q) return fail(AVL_EINVAL, "avl_trajectories_smooth: deposit_q is NULL");
    if ((flags & ~AVL_SMOOTH_VELOCITY) != 0u) return fail(AVL_EINVAL, "avl_trajectories_smooth: unknown flag");
    const bool vel = (flags & AVL_SMOOTH_VELOCITY) != 0u;
    if (vel && !velocity_q) return fail(AVL_EINVAL, "avl_trajectories_smooth: velocity_q is NULL");
    const int64_t n = (int64_t)H * W;
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::SmoothWs sw;
    avl::smooth_layout(H, W, max_release_cells, particles_per_cell, step_limit, static_cast<char*>(workspace), &sw);
    avl::SmoothArgs a = smooth_args(dem, mass, H, W, cell_size, params, particles_per_cell, step_limit,
                                    max_release_cells, sw);
    a.dep_q = reinterpret_cast<unsigned long long*>(deposit_q);
    a.vel_q = vel ? reinterpret_cast<unsigned long long*>(velocity_q) : nullptr;
    a.stats = stats ? reinterpret_cast<unsigned long long*>(stats) : sw.w.stats;
    hipError_t e;
    if (!prepared && (e = avl::launch_compact(mask, n, sw.w.cells, sw.w.n_cells, sw.w.blk, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: compaction");
    const avl::RunSpec spec{0u, 0u, 0u, run_id, (unsigned long long)seed};
    if ((e = avl::launch_setup_runs(p_dev ? spec_dev : nullptr, p_dev, p_dev ? 1u : 0u, spec, *params, sw.w.n_cells,
                                    1, 1, 1, H, W, cell_size, particles_per_cell, false, sw.w.runs, sw.w.run_off,
                                    status, s, max_release_cells)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: run setup");
    auto zero = [&]() -> hipError_t {
        hipError_t z;
        if ((z = avl::launch_fill_u32(reinterpret_cast<uint32_t*>(deposit_q), 0u, 2 * n, s)) != hipSuccess) return z;
        if (vel && (z = avl::launch_fill_u32(reinterpret_cast<uint32_t*>(velocity_q), 0u, 2 * n, s)) != hipSuccess)
            return z;
        if ((z = avl::launch_fill_u64(sw.w.queues, 0ull, avl::kXcds * avl::kQueueStride, s)) != hipSuccess) return z;
        return avl::launch_fill_u64(a.stats, 0ull, 4, s);
    };
    if (!prepared && (e = avl::launch_pad_dem(dem, H, W, sw.dem_pad, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: padded DEM");
    if (!prepared &&
        ((e = avl::launch_start_records(dem, H, W, 1, sw.w.cells, sw.w.n_cells, max_release_cells, sw.starts, s)) !=
             hipSuccess ||
         (e = avl::launch_particle_mass(mass, sw.w.cells, sw.w.n_cells, max_release_cells, particles_per_cell,
                                        sw.mpc, s)) != hipSuccess))
        return hip_fail(e, "avl_trajectories_smooth: start records");
    int variant = 0;
    if ((e = choose_smooth(smooth_key(2, n, max_release_cells, particles_per_cell, step_limit),
                           avl::smooth_forward_variants(), s, zero,
                           [&](int v) { return avl::launch_smooth_forward(a, v, s); }, &variant)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: autotune");
    if ((e = zero()) != hipSuccess) return hip_fail(e, "avl_trajectories_smooth: zero");
    if ((e = avl::launch_smooth_forward(a, variant, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: launch");
    if (deposit && (e = avl::launch_q_to_float(a.dep_q, n, deposit, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: deposit");
    if (vel && velocity && (e = avl::launch_q_to_float(a.vel_q, n, velocity, s)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_smooth: velocity");
    return AVL_OK;
}
}  // namespace

int avl_trajectories_smooth(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                            float cell_size, const avl_params* params, uint32_t particles_per_cell,
                            uint32_t step_limit, uint64_t seed, uint32_t run_id, int32_t max_release_cells,
                            uint32_t flags, int64_t* deposit_q, float* deposit, int64_t* velocity_q, float* velocity,
                            uint64_t* stats, int32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
    return smooth_forward(dem, mask, mass, H, W, cell_size, params, particles_per_cell, step_limit, seed, run_id,
                          max_release_cells, flags, deposit_q, deposit, velocity_q, velocity, stats, status, workspace,
                          workspace_bytes, stream, false);
}

namespace {
// The adjoint of the pass smooth_forward left in the workspace; p_dev (nullable): xi is read from this device
// copy of the parameters (the loop that keeps them on the device).
int smooth_backward(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                    float cell_size, const avl_params* params, uint32_t particles_per_cell,
                    uint32_t step_limit, int32_t max_release_cells,
                    const float* grad_deposit, double* dparams, float* dmass, float* per_particle,
                    void* workspace, size_t workspace_bytes, void* stream, const avl_params* p_dev) {
    g_last_error.clear();
    int rc = smooth_checks("avl_trajectories_backward", dem, mask, H, W, cell_size, params, particles_per_cell,
                           step_limit, max_release_cells, workspace, workspace_bytes);
    if (rc != AVL_OK) return rc;
    if (!grad_deposit || !dparams || !dmass) return fail(AVL_EINVAL, "avl_trajectories_backward: null pointer");
    const int64_t n = (int64_t)H * W;
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::SmoothWs sw;
    avl::smooth_layout(H, W, max_release_cells, particles_per_cell, step_limit, static_cast<char*>(workspace), &sw);
    avl::SmoothArgs a = smooth_args(dem, mass, H, W, cell_size, params, particles_per_cell, step_limit,
                                    max_release_cells, sw);
    a.gD = grad_deposit;
    a.pdev = p_dev;
    hipError_t e;
    auto zero = [&]() -> hipError_t {
        hipError_t z;
        if ((z = avl::launch_fill_u32(reinterpret_cast<uint32_t*>(dmass), 0u, n, s)) != hipSuccess) return z;
        return avl::launch_fill_u64(sw.w.queues, 0ull, avl::kXcds * avl::kQueueStride, s);
    };
    int variant = 0;
    if ((e = choose_smooth(smooth_key(3, n, max_release_cells, particles_per_cell, step_limit),
                           avl::smooth_backward_variants(), s, zero,
                           [&](int v) { return avl::launch_smooth_backward_kernel(a, v, s); }, &variant)) !=
        hipSuccess)
        return hip_fail(e, "avl_trajectories_backward: autotune");
    if ((e = zero()) != hipSuccess) return hip_fail(e, "avl_trajectories_backward: zero");
    if ((e = avl::launch_smooth_backward_kernel(a, variant, s)) != hipSuccess ||
        (e = avl::launch_smooth_reductions(a, sw.w.n_cells, dmass, max_release_cells, sw.part, dparams, s)) !=
            hipSuccess)
        return hip_fail(e, "avl_trajectories_backward: launch");
    if (per_particle && a.cap &&
        (e = hipMemcpyAsync(per_particle, sw.pp, 4 * (size_t)a.cap * sizeof(float), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
        return hip_fail(e, "avl_trajectories_backward: copy");
    return AVL_OK;
}
}  // namespace

int avl_trajectories_backward(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                              float cell_size, const avl_params* params, uint32_t particles_per_cell,
                              uint32_t step_limit, uint64_t seed, uint32_t run_id, int32_t max_release_cells,
                              const float* grad_deposit, double* dparams, float* dmass, float* per_particle,
                              void* workspace, size_t workspace_bytes, void* stream) {
    (void)seed;
    (void)run_id;
    return smooth_backward(dem, mask, mass, H, W, cell_size, params, particles_per_cell, step_limit,
                           max_release_cells, grad_deposit, dparams, dmass, per_particle, workspace, workspace_bytes,
                           stream, nullptr);
}

int avl_trajectories_batched(const float* dems, int32_t n_tiles, const uint8_t* masks, int32_t n_masks, int32_t H,
                             int32_t W, float cell_size, const avl_params* params, int32_t n_params,
                             const avl_run* runs, int32_t n_runs, uint32_t particles_per_cell, uint32_t step_limit,
                             uint32_t* counts, float* vmax, uint64_t* stats, int32_t* run_status, void* workspace,
                             size_t workspace_bytes, void* stream) {
    g_last_error.clear();
    static_assert(sizeof(avl_run) == sizeof(avl::RunSpec), "avl_run layout");
    if (!dems || !masks || !params || !runs || !counts || !vmax || !workspace)
        return fail(AVL_EINVAL, "avl_trajectories_batched: null pointer");
    if (!grid_ok(H, W, 1)) return fail(AVL_EINVAL, "avl_trajectories_batched: need H, W >= 1 and H*W < 2^31");
    // the padded patch's row offset is a 24-bit product (W + 2 < 2^24), and positions are binary32
    if (H >= (1 << 23) || W >= (1 << 23)) return fail(AVL_EINVAL, "avl_trajectories_batched: need H, W < 2^23");
    if (n_tiles < 1 || n_masks < 1 || n_params < 1 || n_runs < 1)
        return fail(AVL_EINVAL, "avl_trajectories_batched: need n_tiles, n_masks, n_params, n_runs >= 1");
    const int64_t n = (int64_t)H * W;
    const int64_t lim = (int64_t)0xFFFFFFFFll;
    if ((int64_t)n_runs * n >= lim || (int64_t)n_tiles * n >= lim || (int64_t)n_masks * n >= lim)
        return fail(AVL_EINVAL, "avl_trajectories_batched: n_runs*H*W, n_tiles*H*W, n_masks*H*W must be < 2^32 - 1");
    if (!finite(cell_size) || !(cell_size > 0.0f))
        return fail(AVL_EINVAL, "avl_trajectories_batched: cell_size must be > 0");
    if (particles_per_cell == 0) return fail(AVL_EINVAL, "avl_trajectories_batched: particles_per_cell must be >= 1");
    const int64_t np = avl::padded_cells(H, W);
    if (np >= (int64_t(1) << 30) || (int64_t)n_tiles * np >= lim)
        return fail(AVL_EINVAL, "avl_trajectories_batched: need (H + 2)(W + 2) < 2^30 and n_tiles (H + 2)(W + 2) < 2^32 - 1");
    if (workspace_bytes < avl::batched_workspace_bytes(H, W, n_tiles, n_masks, n_runs))
        return fail(AVL_ENOMEM, "avl_trajectories_batched: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    avl::Workspace ws = avl::carve_batched(workspace, H, W, n_masks, n_runs);

    avl::TrajArgs a{};
    a.dem = dems;
    a.cells = ws.cells;
    a.runs = ws.runs;
    a.run_off = ws.run_off;
    a.queues = ws.queues;
    a.counts = counts;
    a.vmax2 = reinterpret_cast<uint32_t*>(vmax);
    a.stats = stats ? reinterpret_cast<unsigned long long*>(stats) : ws.stats;
    a.H = H;
    a.W = W;
    a.n_runs = (uint32_t)n_runs;
    a.S = step_limit;
    a.g2 = 9.81f + 9.81f;
    a.starts = ws.starts;
    a.pdiv = avl::make_divu32(particles_per_cell);
    a.wdiv = avl::make_divu32((uint32_t)W);
    a.dem_pad = ws.dem_pad;
    a.pad_bytes = (uint32_t)(np * sizeof(float));
    const int64_t raster = (int64_t)n_runs * n;

    auto zero = [&]() -> hipError_t {
        hipError_t e;
        if ((e = avl::launch_fill_u32(counts, 0u, raster, s)) != hipSuccess) return e;
        if ((e = avl::launch_fill_u32(a.vmax2, 0u, raster, s)) != hipSuccess) return e;
        if ((e = avl::launch_fill_u64(ws.queues, 0ull, avl::kXcds * avl::kQueueStride, s)) != hipSuccess) return e;
        return avl::launch_fill_u64(a.stats, 0ull, 4 * (int64_t)n_runs, s);
    };
    // padded copies of the tiles, release-cell lists of every scenario, then the run table
    auto prologue = [&]() -> hipError_t {
        hipError_t e;
        for (int32_t t = 0; t < n_tiles; ++t)
            if ((e = avl::launch_pad_dem(dems + (size_t)t * n, H, W, ws.dem_pad + (size_t)t * np, s)) != hipSuccess)
                return e;
        for (int32_t m = 0; m < n_masks; ++m)
            if ((e = avl::launch_compact(masks + (size_t)m * n, n, ws.cells + (size_t)m * n, ws.n_cells + m, ws.blk,
                                         s)) != hipSuccess)
                return e;
        const avl::RunSpec none{};
        const avl_params none_p{};
        if ((e = avl::launch_fill_u32(reinterpret_cast<uint32_t*>(ws.rec_run), 0x7FFFFFFFu, n_masks, s)) != hipSuccess)
            return e;
        if ((e = avl::launch_setup_runs(reinterpret_cast<const avl::RunSpec*>(runs), params, (uint32_t)n_params, none,
                                        none_p, ws.n_cells, (uint32_t)n_masks, (uint32_t)n_tiles, (uint32_t)n_runs, H,
                                        W, cell_size, particles_per_cell, true, ws.runs, ws.run_off, run_status, s, -1,
                                        ws.rec_run)) != hipSuccess)
            return e;
        return avl::launch_batch_records(reinterpret_cast<const avl::RunSpec*>(runs), ws.rec_run, ws.n_cells,
                                         (uint32_t)n_masks, ws.cells, ws.dem_pad, H, W, ws.starts, s);
    };
    auto body = [&](const avl::LaunchShape& shape) -> hipError_t {
        hipError_t e;
        if ((e = prologue()) != hipSuccess) return e;
        if ((e = zero()) != hipSuccess) return e;
        if ((e = timed_launch(a, true, shape, s)) != hipSuccess) return e;
        return avl::launch_finalize_vmax(a.vmax2, raster, s);
    };

    // the variant is chosen eagerly, before any capture (tuning runs need the run table in place)
    hipError_t e;
    int variant = 0;
    const std::vector<int64_t> tkey = tune_key(true, n, n_runs, particles_per_cell, step_limit);
    bool known = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        known = g_variant_override >= 0 || g_best.count(tkey) != 0;
    }
    if (!known && !capturing(s)) {
        if ((e = prologue()) != hipSuccess) return hip_fail(e, "avl_trajectories_batched: setup");
    }
    if ((e = choose_variant(a, true, tkey, s, zero, &variant)) != hipSuccess)
        return hip_fail(e, "avl_trajectories_batched: autotune");
    g_last_variant = variant;
    const avl::LaunchShape shape = avl::trajectory_shape(true, variant);  // queried outside any capture

    bool use_graph;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        use_graph = g_graphs && s != nullptr;
    }
    if (!use_graph || capturing(s)) {
        e = body(shape);
        return e == hipSuccess ? AVL_OK : hip_fail(e, "avl_trajectories_batched");
    }

    int dev = 0;
    (void)hipGetDevice(&dev);
    uint32_t cs_bits;
    std::memcpy(&cs_bits, &cell_size, 4);
    const std::vector<uint64_t> key{
        (uint64_t)dev, (uint64_t)(uintptr_t)s, (uint64_t)(uintptr_t)dems, (uint64_t)n_tiles, (uint64_t)(uintptr_t)masks,
        (uint64_t)n_masks, (uint64_t)H, (uint64_t)W, cs_bits, (uint64_t)(uintptr_t)params, (uint64_t)n_params,
        (uint64_t)(uintptr_t)runs, (uint64_t)n_runs, particles_per_cell, step_limit, (uint64_t)(uintptr_t)counts,
        (uint64_t)(uintptr_t)vmax, (uint64_t)(uintptr_t)stats, (uint64_t)(uintptr_t)run_status,
        (uint64_t)(uintptr_t)workspace, (uint64_t)variant};
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graph_cache.find(key);
    if (it == g_graph_cache.end()) {
        if (g_graph_cache.size() >= kMaxGraphs) {
            auto old = g_graph_cache.begin();
            for (auto j = g_graph_cache.begin(); j != g_graph_cache.end(); ++j)
                if (j->second.last_use < old->second.last_use) old = j;
            (void)hipGraphExecDestroy(old->second.exec);
            g_graph_cache.erase(old);
        }
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "avl_trajectories_batched: begin capture");
        const hipError_t eb = body(shape);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (eb != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(eb, "avl_trajectories_batched: capture");
        }
        if (e != hipSuccess) return hip_fail(e, "avl_trajectories_batched: end capture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "avl_trajectories_batched: instantiate");
        it = g_graph_cache.emplace(key, GraphEntry{exec, 0}).first;
    }
    it->second.last_use = ++g_clock;
    if ((e = hipGraphLaunch(it->second.exec, s)) != hipSuccess) return hip_fail(e, "avl_trajectories_batched: launch");
    return AVL_OK;
}

// ------------------------------------------------------------------ calibration loop
namespace {

struct CalibWs {
    char* smooth;      // the smooth pass's own workspace (checkpoints for the adjoint)
    size_t smooth_bytes;
    int64_t* dep_q;    // H*W
    float* dep;        // H*W
    float* gD;         // H*W
    float* dmass;      // H*W
    double* part;      // loss partial sums
    double* scal;      // [loss, dL/dmu, dL/dxi, dL/dh]
    int32_t* status;   // smooth pass status
    avl::RunSpec* spec;  // the run, on the device
    avl_params* p;       // the current parameters, on the device
    double* state;       // Adam's state (avl::kCalibState)
    double* hist;        // kCalibRows history rows of 5, copied to the caller's history as they fill
    int32_t* err;        // (first nonzero status, its iteration)
};
constexpr int32_t kCalibRows = 64;

size_t calib_layout(int32_t H, int32_t W, int32_t max_cells, uint32_t P, uint32_t S, char* base, CalibWs* c) {
    const int64_t n = (int64_t)H * W;
    const size_t sm = avl::round256(avl_smooth_workspace_bytes(H, W, max_cells, P, S));
    size_t off = sm;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += avl::round256(bytes);
        return p;
    };
    char* dq = take((size_t)n * 8);
    char* d = take((size_t)n * 4);
    char* g = take((size_t)n * 4);
    char* dm = take((size_t)n * 4);
    char* pt = take(avl::mse_partials() * sizeof(double));
    char* sc = take(4 * sizeof(double) + sizeof(int32_t));
    char* spc = take(sizeof(avl::RunSpec));
    char* pp = take(sizeof(avl_params));
    char* stt = take(avl::kCalibState * sizeof(double));
    char* hs = take((size_t)kCalibRows * 5 * sizeof(double));
    char* er = take(2 * sizeof(int32_t));
    if (c) {
        c->smooth = base;
        c->smooth_bytes = sm;
        c->dep_q = reinterpret_cast<int64_t*>(dq);
        c->dep = reinterpret_cast<float*>(d);
        c->gD = reinterpret_cast<float*>(g);
        c->dmass = reinterpret_cast<float*>(dm);
        c->part = reinterpret_cast<double*>(pt);
        c->scal = reinterpret_cast<double*>(sc);
        c->status = reinterpret_cast<int32_t*>(sc + 4 * sizeof(double));
        c->spec = reinterpret_cast<avl::RunSpec*>(spc);
        c->p = reinterpret_cast<avl_params*>(pp);
        c->state = reinterpret_cast<double*>(stt);
        c->hist = reinterpret_cast<double*>(hs);
        c->err = reinterpret_cast<int32_t*>(er);
    }
    return off;
}

}  // namespace

size_t avl_calibrate_workspace_bytes(int32_t H, int32_t W, int32_t max_release_cells, uint32_t particles_per_cell,
                                     uint32_t step_limit) {
    if (avl_smooth_workspace_bytes(H, W, max_release_cells, particles_per_cell, step_limit) == 0) return 0;
    return calib_layout(H, W, max_release_cells, particles_per_cell, step_limit, nullptr, nullptr);
}

int avl_calibrate(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W, float cell_size,
                  const avl_params* start, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                  uint32_t run_id, int32_t max_release_cells, const float* target, int32_t n_iters,
                  const avl_adam* adam, double* history, avl_params* result, void* workspace, size_t workspace_bytes,
                  void* stream) {
    g_last_error.clear();
    const char* where = "avl_calibrate";
    if (!target || !adam || !result || !workspace || !start) return fail(AVL_EINVAL, "%s: null pointer", where);
    if (n_iters < 0) return fail(AVL_EINVAL, "%s: n_iters must be >= 0", where);
    if (n_iters > 0 && !history) return fail(AVL_EINVAL, "%s: history is NULL", where);
    if (!(finite(adam->lr_mu) && adam->lr_mu > 0.0f && finite(adam->lr_xi) && adam->lr_xi > 0.0f))
        return fail(AVL_EINVAL, "%s: step sizes must be finite and > 0", where);
    if (!(adam->beta1 >= 0.0f && adam->beta1 < 1.0f && adam->beta2 >= 0.0f && adam->beta2 < 1.0f))
        return fail(AVL_EINVAL, "%s: need 0 <= beta1, beta2 < 1", where);
    if (!(finite(adam->eps) && adam->eps > 0.0f)) return fail(AVL_EINVAL, "%s: eps must be finite and > 0", where);
    if (!(finite(adam->mu_min) && adam->mu_min >= 0.0f && finite(adam->xi_min) && adam->xi_min > 0.0f))
        return fail(AVL_EINVAL, "%s: need finite mu_min >= 0 and xi_min > 0", where);
    if (!finite(start->xi)) return fail(AVL_EINVAL, "%s: the start xi must be finite", where);
    if (workspace_bytes < avl_calibrate_workspace_bytes(H, W, max_release_cells, particles_per_cell, step_limit))
        return fail(AVL_ENOMEM, "%s: workspace too small", where);
    CalibWs c;
    calib_layout(H, W, max_release_cells, particles_per_cell, step_limit, static_cast<char*>(workspace), &c);
    int rc = smooth_checks(where, dem, mask, H, W, cell_size, start, particles_per_cell, step_limit,
                           max_release_cells, c.smooth, c.smooth_bytes);
    if (rc != AVL_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = (int64_t)H * W;
    const float cgrad = 2.0f / (float)n;
    // The loop stays on the device: the run constants are set up from a device copy of the parameters, the
    // adjoint reads xi from it, and a one-thread kernel takes the Adam step in binary64 (the same arithmetic
    // in the same order as a host loop would) and writes the history row. The host only enqueues; rows come
    // back in blocks of kCalibRows, and a nonzero status of any pass is reported after the loop.
    avl::AdamConsts ac;
    ac.lr[0] = (double)adam->lr_mu;
    ac.lr[1] = (double)adam->lr_xi;
    ac.b1 = adam->beta1;
    ac.b2 = adam->beta2;
    ac.eps = adam->eps;
    ac.lo[0] = (double)adam->mu_min;
    ac.lo[1] = (double)adam->xi_min;
    const avl::RunSpec spec{0u, 0u, 0u, run_id, (unsigned long long)seed};
    hipError_t e = avl::launch_calib_init(spec, *start, c.spec, c.p, c.state, c.err, s);
    if (e != hipSuccess) return hip_fail(e, "avl_calibrate: init");
    // an error inside the loop returns only after the stream has drained: history rows copied earlier in
    // the loop may still be on their way into the caller's buffer
    auto drained = [&](int code) {
        (void)hipStreamSynchronize(s);
        return code;
    };
    for (int32_t t = 0; t < n_iters; ++t) {
        // after the first pass the release cells, padded DEM, start records and masses are in the workspace
        if ((rc = smooth_forward(dem, mask, mass, H, W, cell_size, start, particles_per_cell, step_limit, seed,
                                 run_id, max_release_cells, 0u, c.dep_q, c.dep, nullptr, nullptr, nullptr, c.status,
                                 c.smooth, c.smooth_bytes, stream, t > 0, c.p, c.spec)) != AVL_OK)
            return drained(rc);
        if ((e = avl::launch_mse_grad(c.dep, target, n, cgrad, c.gD, c.part, c.scal, s)) != hipSuccess)
            return drained(hip_fail(e, "avl_calibrate: loss"));
        if ((rc = smooth_backward(dem, mask, mass, H, W, cell_size, start, particles_per_cell, step_limit,
                                  max_release_cells, c.gD, c.scal + 1, c.dmass, nullptr, c.smooth, c.smooth_bytes,
                                  stream, c.p)) != AVL_OK)
            return drained(rc);
        const int32_t slot = t % kCalibRows;
        if ((e = avl::launch_adam_step(c.scal, c.status, c.state, c.p, c.hist + 5 * slot, ac, t, c.err, s)) !=
            hipSuccess)
            return drained(hip_fail(e, "avl_calibrate: step"));
        if (slot == kCalibRows - 1 || t == n_iters - 1) {
            // stream-ordered before the next step overwrites the rows
            if ((e = hipMemcpyAsync(history + 5 * (int64_t)(t - slot), c.hist, (size_t)(slot + 1) * 5 * sizeof(double),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
                return drained(hip_fail(e, "avl_calibrate: history"));
        }
    }
    struct {
        double st[avl::kCalibState];
        int32_t err[2];
    } h{};
    h.st[0] = (double)start->mu;
    h.st[1] = (double)start->xi;
    if (n_iters > 0 &&
        ((e = hipMemcpyAsync(h.st, c.state, sizeof(h.st), hipMemcpyDeviceToHost, s)) != hipSuccess ||
         (e = hipMemcpyAsync(h.err, c.err, sizeof(h.err), hipMemcpyDeviceToHost, s)) != hipSuccess ||
         (e = hipStreamSynchronize(s)) != hipSuccess))
        return drained(hip_fail(e, "avl_calibrate: read back"));
    if (h.err[0] == 3)
        return fail(AVL_EINVAL, "%s: the mask has more release cells than max_release_cells", where);
    if (h.err[0] != 0)
        return fail(AVL_EINVAL, "%s: the parameters of iteration %d are invalid (status %d)", where, h.err[1],
                    h.err[0]);
    const double th[2] = {h.st[0], h.st[1]};
    *result = *start;
    result->mu = (float)th[0];
    result->xi = (float)th[1];
    return AVL_OK;
}


}  // extern "C"
