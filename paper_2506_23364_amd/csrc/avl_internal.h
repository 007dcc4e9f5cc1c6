// Internal declarations shared by the libavl translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/avl.h"

#include <cstddef>
#include <cstdint>

namespace avl {

constexpr int kWave = 64;

// ------------------------------------------------------------------ workspace layout
// Single run (avl_workspace_bytes):
//   [0, kControl) control block: n_cells (i32 @0), stats (4 x u64 @64), run offsets (2 x u64 @192), the
//                run's constants (RunConst @256), per-XCD slot queues (kXcds u64 @512, kQueueStride words
//                apart)
//   then         per-block sums of the compaction scan (u32), the release-texel list (i32, one per texel of
//                the release texture: mult^2 H W), the start records of the release texels (StartRec, as
//                many) and the padded DEM (f32, (H + 2) x (W + 2))
// Batch (avl_batched_workspace_bytes):
//   [0, kControl) control block: per-XCD slot queues @512, kQueueStride words apart
//   then         compaction scan sums; n_masks release-cell lists (i32, H*W each); n_masks cell counts;
//                n_runs RunConst; n_runs + 1 slot offsets; n_runs x 4 internal statistics; n_tiles padded
//                DEM tiles (f32, (H + 2) x (W + 2) each)
// Every region starts on a 256-byte boundary.
constexpr int kXcds = 8;            // MI355X: 8 XCDs, each with its own L2
// The slot queues' counters sit 256 bytes apart: device-scope atomics are performed at the memory side
// and serialise per memory line, and with the eight counters in one line every wave's take from the
// queues waited for the other XCDs' takes as well (4.5-10 us per take in the smooth kernels).
constexpr uint32_t kQueueStride = 32;
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanChunk = kScanThreads * kScanPerThread;  // cells per compaction block
constexpr size_t kControl = 512 + (size_t)kXcds * kQueueStride * 8;

inline size_t round256(size_t v) { return (v + 255) & ~size_t(255); }
inline int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

struct RunConst;
struct StartRec;

struct Workspace {
    int32_t* n_cells;             // single: 1; batch: n_masks
    unsigned long long* queues;   // kXcds counters, kQueueStride words apart
    unsigned long long* stats;    // single: 4; batch: 4 x n_runs
    unsigned long long* run_off;  // n_runs + 1
    RunConst* runs;               // n_runs
    uint32_t* blk;
    int32_t* cells;               // single: mult^2 H W; batch: n_masks x H*W
    StartRec* starts;             // single: mult^2 H W; batch: n_masks x H*W, parallel to cells
    int32_t* rec_run;             // batch only: per scenario, the first valid run that uses it
    float* dem_pad;               // single: (H + 2) x (W + 2); batch: n_tiles of them
};

// cells of the DEM with a one-texel border
__host__ __device__ inline int64_t padded_cells(int64_t H, int64_t W) { return (H + 2) * (W + 2); }
size_t workspace_bytes(int64_t H, int64_t W, int64_t mult = 1);   // mult: release texels per DEM cell edge
Workspace carve(void* base, int64_t H, int64_t W, int64_t mult = 1);
size_t batched_workspace_bytes(int64_t H, int64_t W, int64_t n_tiles, int64_t n_masks, int64_t n_runs);
Workspace carve_batched(void* base, int64_t H, int64_t W, int64_t n_masks, int64_t n_runs);

// ------------------------------------------------------------------ trajectory kernel arguments
// Derived constants of one run (one parameter set on one DEM tile and release scenario), binary32,
// computed on the device by k_setup_runs in the model's order.
struct RunConst {
    float per, Q, rnd, L;      // persistence, 1 - persistence, randomness, step length (cells)
    float dl2, mdl, cd, tca;   // (L cs)^2, mu L cs, 2g / (xi h), tan(alpha) cs
    uint32_t key0, key1;       // Philox key = 64-bit seed
    uint32_t run, use_alpha;   // Philox counter word 3; runout-angle stop on/off
    uint32_t dem_off;          // element offset of the run's DEM tile
    uint32_t cells_off;        // element offset of the run's release-cell list
    uint32_t raster_off;       // element offset of the run's rasters
    uint32_t P;                // particles per release cell
    unsigned long long n_slots;  // release cells x P
    uint32_t pad_off;          // element offset of the run's padded DEM tile
    uint32_t use_rec;          // batch: its scenario's start records were made on its tile
};
static_assert(sizeof(RunConst) == 80, "RunConst layout");

// Start state of the particles released at one cell (the cell centre, its bilinear sample and the
// downslope unit direction), computed once per release cell for a single run.
struct StartRec {
    float x, y, z, gx, gy, dx, dy;
    uint32_t cell;
};
static_assert(sizeof(StartRec) == 32, "StartRec layout");

// Unsigned 32-bit division by an invariant d >= 1 (Granlund and Montgomery, PLDI 1994, section 4):
// q = (t + ((n - t) >> sh1)) >> sh2 with t = mulhi(mul, n), exact for every 32-bit n.
struct DivU32 {
    uint32_t mul, sh1, sh2;
};
inline DivU32 make_divu32(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;  // l = ceil(log2 d)
    DivU32 v;
    v.mul = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    v.sh1 = l < 1 ? l : 1;
    v.sh2 = l > 1 ? l - 1 : 0;
    return v;
}

struct TrajArgs {
    const float* __restrict__ dem;               // all DEM tiles, H*W each
    const int32_t* __restrict__ cells;           // all release-cell lists, H*W each
    const RunConst* __restrict__ runs;           // n_runs
    const unsigned long long* __restrict__ run_off;  // n_runs + 1 slot offsets, each a multiple of 64
    unsigned long long* __restrict__ queues;     // kXcds slot counters kQueueStride words apart, zero at launch
    uint32_t* __restrict__ counts;               // count rasters, zero at launch
    uint32_t* __restrict__ vmax2;                // binary32 bits of the per-cell max of v^2 (v^2 >= 0, so bit
                                                 // order is value order), zero at launch
    unsigned long long* __restrict__ stats;      // 4 u64 per run: steps, exits, stops, step-limit ends
    int32_t H, W;
    uint32_t n_runs;
    uint32_t S;                                  // step limit
    float g2;                                    // 2g
    const StartRec* __restrict__ starts;         // single run: one per release cell; batched: NULL
    DivU32 pdiv;                                 // division by the particles per cell (same for every run)
    const float* __restrict__ dem_pad;           // the DEM tiles with a replicated border, (H + 2)(W + 2) each
    uint32_t pad_bytes;                          // bytes of one padded tile, (H + 2) (W + 2) x 4 < 2^32
    uint32_t runout_angle;                       // single run: 1 if it uses the runout-angle stop (selects the
                                                 // kernel instantiation; a batch always has the stop compiled in)
    DivU32 wdiv;                                 // division by W (a batch's release cell -> row, column)
    // path recording (single run, the recording instantiation only): particles [rec_first, rec_first +
    // rec_n) of the run write their end record and, with rec_xy, their points (the release point, the
    // position after every accepted step, and an energy or runout-angle stop's rejected target)
    unsigned long long rec_first;
    uint32_t rec_n;
    uint32_t rec_stride;                         // points per particle without rec_off
    const unsigned long long* __restrict__ rec_off;  // nullable: first point of each recorded particle
    float2* __restrict__ rec_xy;                 // nullable: the points
    float* __restrict__ rec_v2;                  // nullable: v^2 at each point (0 at the release point and
                                                 // at a rejected target)
    uint32_t* __restrict__ rec_end;              // (accepted steps << 2) | end (0 limit, 1 exit, 2 stop)
    uint32_t slots_per_lane;                     // sizes a small problem's grid (set from the kernel variant)
    unsigned long long* __restrict__ probe;      // nullable: 3 per block, the real-time clock at the block's
                                                 // start, when it runs out of slots, and at its end
};

struct LaunchShape {
    int block;  // threads per block (multiple of 64)
    int grid;   // blocks
    int variant;  // kernel variant index (see trajectory_variants)
};

// ------------------------------------------------------------------ launchers (enqueue only; return hipError_t)
hipError_t launch_normals(const float* dem, int H, int W, float cs, float* out4, hipStream_t s);
// normals and the release map of the same texels in one pass (cmin, cmax: the cosines of the slope range)
hipError_t launch_normals_mask(const float* dem, int H, int W, float cs, float cmin, float cmax, float zmin,
                               float zmax, float* out4, uint8_t* mask, hipStream_t s);
hipError_t launch_release_mask(const float* normals4, const float* dem, int64_t n, float cmin, float cmax,
                               float zmin, float zmax, uint8_t* mask, hipStream_t s);
hipError_t launch_snow_cover(const float* normals4, const float* dem, int64_t n, float z_lo, float z_hi, float c_lo,
                             float c_hi, float* alpha, hipStream_t s);
hipError_t launch_release_mask_fine(const float* normals4, const float* dem, int H, int W, int mult, float cmin,
                                    float cmax, float zmin, float zmax, uint8_t* mask, hipStream_t s);
hipError_t launch_compact(const uint8_t* mask, int64_t n, int32_t* cells, int32_t* n_cells, uint32_t* blk,
                          hipStream_t s);
// Overlay mipmap: up to kMipPass output levels per pass (a 32 x 32 tile of the first halves to 1 x 1).
constexpr int kMipPass = 6;
struct MipLevels {
    unsigned long long* c[kMipPass];
    float* v[kMipPass];
    int h[kMipPass], w[kMipPass];
};
hipError_t launch_mip_pass(const void* cin, bool cin64, const float* vin, int h0, int w0, int nlev,
                           const MipLevels& o, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);
// (H + 2) x (W + 2) copy of the DEM with the edge texels replicated into a one-texel border.
hipError_t launch_pad_dem(const float* dem, int H, int W, float* out, hipStream_t s);
// starts[i] for each of the first min(*n_cells, n) release cells (the records array holds n).
hipError_t launch_start_records(const float* dem, int H, int W, int mult, const int32_t* cells,
                                const int32_t* n_cells, int64_t n, StartRec* starts, hipStream_t s);
// Setup of the run table: per run, constants from its parameter set and the slot count from its
// scenario's release-cell count (written by the compaction); then 64-aligned slot offsets.
struct RunSpec {
    uint32_t tile, scenario, param, run_id;
    unsigned long long seed;
};
// specs/params: device arrays (batched) or NULL, then one_spec/one_param are used for the single run.
// cap_cells >= 0: a run whose scenario has more release cells than cap_cells gets no slots (status 3).
// rec_run (batched, n_scen entries filled with INT32_MAX beforehand, or NULL): receives per scenario the
// lowest valid run index that uses it; a run whose tile is that run's tile gets use_rec = 1.
hipError_t launch_setup_runs(const RunSpec* specs, const ::avl_params* params, uint32_t n_params, RunSpec one_spec,
                             ::avl_params one_param, const int32_t* n_cells_per_scen, uint32_t n_scen, uint32_t n_tiles,
                             uint32_t n_runs, int32_t H, int32_t W, float cell_size, uint32_t P, bool batched,
                             RunConst* runs, unsigned long long* run_off, int32_t* status, hipStream_t s,
                             int64_t cap_cells = -1, int32_t* rec_run = nullptr);
// Batch: start records of every scenario's release cells on the tile of the scenario's first valid run
// (rec_run from the run setup), read from the padded tiles; starts and cells are n_scen x HW arrays.
hipError_t launch_batch_records(const RunSpec* specs, const int32_t* rec_run, const int32_t* n_cells_per_scen,
                                uint32_t n_scen, const int32_t* cells, const float* dem_pad, int32_t H, int32_t W,
                                StartRec* starts, hipStream_t s);
hipError_t launch_trajectories(const TrajArgs& a, bool batched, const LaunchShape& shape, hipStream_t s);
// The recording instantiation (single run, variant 0's shape, runout-angle stop compiled in).
hipError_t launch_trajectories_record(const TrajArgs& a, hipStream_t s);

// Memory microbenchmarks (membench.hip): the wave-order schedule of a recorded pass's gathers and cell visits,
// the replays of both, and a copy.
hipError_t launch_replay_schedule(int mode, const float2* pts, const float* v2s, const unsigned long long* off,
                                  const uint32_t* ends, uint64_t n, int W, unsigned long long* totals,
                                  const unsigned long long* gbase, const unsigned long long* vbase, uint32_t* gathers,
                                  uint2* visits, hipStream_t s);
hipError_t launch_replay_gather(const uint32_t* sched, uint64_t n, const float* dem_pad, uint32_t pad_bytes,
                                uint32_t row_bytes, uint32_t* checksum, hipStream_t s);
hipError_t launch_replay_atomics(const uint2* sched, uint64_t n, uint32_t* counts, uint32_t* vmax2, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, uint64_t n16, hipStream_t s);

// Smooth forward and adjoint (smooth.hip)
struct SmoothArgs {
    const float* dem;
    const float* mass;         // nullable: 1 per release cell
    const int32_t* cells;
    const RunConst* runs;      // one run
    const unsigned long long* run_off;
    unsigned long long* queues;  // kXcds slot counters kQueueStride words apart, zero at launch
    unsigned long long* dep_q;
    unsigned long long* vel_q;  // nullable
    unsigned long long* stats;
    float* ck;                 // 5 x C x cap checkpoints (x, y, dx, dy, v^2), SoA
    uint32_t* end_rec;         // cap: steps done << 2 | end reason
    const float* gD;           // adjoint: dL/dD
    float* pp;                 // adjoint: 4 x cap per-particle results (dmu, dxi, dh, sum gD w)
    float2* scratch;           // adjoint: kCkpt x (grid threads) of (a_k, v^2_{k+1})
    int32_t H, W;
    uint32_t S, C;                          // step limit, checkpoints per particle
    unsigned long long cap;                 // particle capacity of ck / end_rec / pp
    float g2, g2dl, xi, h;                  // 2g, 2g * dl (dl = step_cells * cell_size), xi, h
    const float* dem_pad;                   // the DEM with a replicated border, (H + 2) x (W + 2)
    uint32_t pad_bytes;                     // its bytes, < 2^32
    uint32_t spl;                           // particle slots per lane of a small problem (set by the launchers)
    const StartRec* starts;                 // per release cell: the start state of its particles
    const float* mpc;                       // per release cell: the mass of each of its particles
    DivU32 pdiv;                            // slot -> release cell (division by the particles per cell)
    const ::avl_params* pdev;               // nullable: the adjoint reads xi here (a device-side loop) not from .xi
};


size_t smooth_checkpoints(uint32_t S);
size_t smooth_scratch_bytes();
size_t smooth_reduce_blocks(unsigned long long cap);
// Kernel variants of the smooth forward and of the adjoint (grid shapes only: every variant gives the same
// results); the library's tuner picks one per problem size.
int smooth_forward_variants();
int smooth_backward_variants();
hipError_t launch_smooth_forward(const SmoothArgs& a, int variant, hipStream_t s);
hipError_t launch_smooth_backward_kernel(const SmoothArgs& a, int variant, hipStream_t s);
// the adjoint's reductions after its kernel: dL/dparams and dL/dmass
hipError_t launch_smooth_reductions(const SmoothArgs& a, const int32_t* n_cells, float* dmass, int64_t n_grid,
                                    double* part, double* dparams, hipStream_t s);
hipError_t launch_q_to_float(const unsigned long long* q, int64_t n, float* out, hipStream_t s);
// per release cell i < *n_cells: mpc[i] = (mass ? mass[cells[i]] : 1) / P, the mass each of its particles carries
hipError_t launch_particle_mass(const float* mass, const int32_t* cells, const int32_t* n_cells, int64_t cap,
                                uint32_t P, float* mpc, hipStream_t s);
// calibration loss: gD = c (D - T) and L = sum (D - T)^2 / N (binary64, fixed order) into *loss
hipError_t launch_mse_grad(const float* dep, const float* target, int64_t n, float c, float* gD, double* part,
                           double* loss, hipStream_t s);
size_t mse_partials();

// Device side of the calibration loop. State: th_mu, th_xi, m_mu, m_xi, v_mu, v_xi, beta1^t, beta2^t (binary64).
struct AdamConsts {
    double lr[2], b1, b2, eps, lo[2];
};
constexpr int kCalibState = 8;
// writes the run spec, the parameters and the initial state (th = the start's mu, xi; m = v = 0; products 1)
hipError_t launch_calib_init(RunSpec spec, ::avl_params start, RunSpec* spec_dev, ::avl_params* p_dev, double* state,
                             int32_t* err, hipStream_t s);
// one Adam step from scal = [loss, dL/dmu, dL/dxi, dL/dh]: writes the history row (loss, mu, xi, dL/dmu, dL/dxi,
// before the step), updates the state and the parameters; the first iteration whose pass reported a nonzero
// status is kept in err = (status, iteration)
hipError_t launch_adam_step(const double* scal, const int32_t* status, double* state, ::avl_params* p_dev,
                            double* row, AdamConsts c, int32_t t, int32_t* err, hipStream_t s);
hipError_t launch_finalize_vmax(uint32_t* vmax_bits, int64_t n, hipStream_t s);

// Persistent-grid shape of kernel variant `variant` on the current device; number of variants.
LaunchShape trajectory_shape(bool batched, int variant);
int trajectory_variants();
// info[0..7]: threads per block, iterations per epoch, table slots, probes, window top-up (x block), retention
// threshold, waves per SIMD of the register budget, slots per lane; false for an index out of range.
bool trajectory_variant_info(int variant, int32_t* info);

}  // namespace avl
