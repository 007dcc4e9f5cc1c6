/*
 * avl.h -- C ABI of libavl.so, the MI355X (gfx950) hot path of the data-driven avalanche overlay of
 * "Data-Driven Compute Overlays for Interactive Geographic Simulation and Visualization"
 * (arXiv 2506.23364), section 5.2 (Avalanches): normals from a DEM, a release-point map from a
 * steepness range, and Monte-Carlo particle trajectories from every release texel, accumulated into a
 * hit-count raster and a per-texel maximum-velocity raster (the velocity indicator of figure 4).
 *
 * Conventions shared by every entry point
 *  - Rasters are row-major H x W (row r, column c at index r*W + c). x runs along columns, y along
 *    rows; texel (r, c) covers [c, c+1) x [r, r+1) in cell units and its height sits at its centre.
 *  - Every array argument is a DEVICE pointer on the current HIP device, allocated and owned by the
 *    caller; the library never frees or keeps a caller pointer past the call. Scalars and the
 *    parameter struct are host values. Outputs are overwritten completely.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). All work is enqueued
 *    asynchronously on it; the call returns after the launches, not after the work.
 *  - Return value: AVL_OK (0) or a negative error code. Arguments are checked on the host before any
 *    launch, so an error leaves every output untouched. avl_strerror() names a code and
 *    avl_last_error() gives the detail of the last failure on the calling thread.
 *  - Arithmetic is IEEE binary32, round to nearest, without contraction, in the order defined for
 *    each call, so that integer results (counts, masks, cell lists) are reproducible bit for bit and
 *    independent of launch shape, block order and XCD.
 *  - Calls are thread-safe; concurrent calls must use distinct workspaces.
 */
#ifndef AVL_H
#define AVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define AVL_API __attribute__((visibility("default")))
#else
#define AVL_API
#endif

#define AVL_OK 0
#define AVL_EINVAL (-1) /* bad argument: null pointer, size, parameter range */
#define AVL_ENOMEM (-2) /* workspace smaller than the size the matching *_workspace_bytes call returns */
#define AVL_EHIP (-3)   /* HIP runtime or launch error; avl_last_error() has the HIP message */

/* Model parameters of the trajectory node (section 5.2: persistence, runout angle, random variation,
 * plus the friction law that turns the path into a speed). */
typedef struct avl_params {
    float mu;          /* Coulomb friction coefficient, finite, >= 0 */
    float xi;          /* Voellmy turbulence coefficient in m/s^2, > 0; +INFINITY = no drag */
    float flow_height; /* flow height h in metres, finite, > 0 */
    float persistence; /* weight of the previous direction, in [0, 1] (the paper's default 0.9) */
    float randomness;  /* amplitude of the random deviation, finite, >= 0 (the paper's default 0.16) */
    float step_cells;  /* horizontal step length in cells, finite, in (0, 16] (default 1) */
    float tan_alpha;   /* runout-angle stop: tan(alpha), finite; any negative value disables it */
    uint32_t flags;    /* must be 0 */
} avl_params;

/* Surface normals and steepness (section 5.2, the normals node; section 5.1 shares it).
 * dem: H*W float heights in metres. cell_size: texel edge in metres, finite, > 0. H, W >= 2.
 * normals4: H*W*4 floats (16-byte aligned), per texel (nx, ny, nz, slope in degrees), with the gradient
 *   gx = (z[r][c+1] - z[r][c-1]) / (2 cs) inside and the one-sided (z[r][1]-z[r][0]) / cs,
 *   (z[r][W-1]-z[r][W-2]) / cs at the left/right edges (gy likewise along rows), l = sqrt(gx^2+gy^2+1),
 *   n = (-(gx/l), -(gy/l), 1/l). The slope channel atan(sqrt(gx^2+gy^2)) in degrees is for display
 *   (within a few ulp of the correctly rounded value); the release mask reads only nz. */
AVL_API int avl_normals(const float* dem, int32_t H, int32_t W, float cell_size, float* normals4, void* stream);

/* Release map (section 5.2, the release-point node: a steepness range per normal texel; an elevation
 * window is added). mask[i] = 1 when cos(smax) <= nz <= cos(smin) and z_min <= dem[i] <= z_max, else 0.
 * The cosines are taken on the host in binary64 from deg * (pi / 180) and rounded once to binary32.
 * normals4 as written by avl_normals; 0 <= slope_min_deg <= slope_max_deg <= 90; z bounds may be
 * +-INFINITY, not NaN. H, W >= 1. mask: H*W bytes. */
AVL_API int avl_release_mask(const float* normals4, const float* dem, int32_t H, int32_t W, float slope_min_deg,
                     float slope_max_deg, float z_min, float z_max, uint8_t* mask, void* stream);

/* Normals and release map in one pass (sections 5.1 and 5.2: the normals node feeding the release-point
 * node): writes exactly what avl_normals followed by avl_release_mask on its normals writes, reading the
 * DEM once and never reading the normals back. Arguments as for those two calls (H, W >= 2, normals4
 * 16-byte aligned, the same slope and elevation bounds and errors); normals4 and mask are outputs. */
AVL_API int avl_normals_release_mask(const float* dem, int32_t H, int32_t W, float cell_size, float slope_min_deg,
                                     float slope_max_deg, float z_min, float z_max, float* normals4, uint8_t* mask,
                                     void* stream);

/* Snow cover (section 5.1: from the terrain alone, with the snow line, the maximal steepness and blend
 * factors for the transition zones as parameters; the overlay is white with the blend factor as alpha).
 * alpha[i] = a_z * a_s in binary32, where a ramp over [lo, hi] is (v - lo) / (hi - lo) clamped to [0, 1]
 * (NaN gives 0), or the step v >= lo when hi <= lo:
 *   a_z: v = dem[i] over [snow_line, snow_line + alt_blend] (the upper end rounded once to binary32);
 *   a_s: v = nz (channel 2 of normals4) over [cos(max_slope), cos(max_slope - slope_blend)], the cosines
 *        taken on the host in binary64 and rounded once (full cover up to max_slope - slope_blend, none
 *        beyond max_slope, linear in nz between).
 * normals4 as written by avl_normals (16-byte aligned); finite snow_line; finite alt_blend >= 0;
 * 0 <= slope_blend_deg <= max_slope_deg <= 90. H, W >= 1. alpha: H*W floats. */
AVL_API int avl_snow_cover(const float* normals4, const float* dem, int32_t H, int32_t W, float snow_line,
                           float alt_blend, float max_slope_deg, float slope_blend_deg, float* alpha, void* stream);

/* Workspace bytes that avl_release_cells and avl_trajectories need for an H x W grid. */
AVL_API size_t avl_workspace_bytes(int32_t H, int32_t W);

/* Release-cell list (particles are released per coded texel, section 5.2): the linear indices r*W+c
 * of the nonzero bytes of mask in row-major order, into cells[0 .. n-1], and n into *n_cells (a device
 * int32). cells must hold H*W entries. workspace: device memory of avl_workspace_bytes(H, W) bytes. */
AVL_API int avl_release_cells(const uint8_t* mask, int32_t H, int32_t W, int32_t* cells, int32_t* n_cells,
                      void* workspace, size_t workspace_bytes, void* stream);

/* Particle trajectories (section 5.2, the trajectory node), one pass over every release texel.
 *
 * From each nonzero texel of mask (H*W bytes), particles_per_cell particles start at the texel
 * centre with speed 0, heading straight downslope; particle (cell, j) draws its random deviation from
 * Philox4x32-10 with counter (step/2, j, cell index r*W+c, run_id) and key (seed low, seed high) words,
 * so its path does not depend on which other texels are released. Per step, in binary32:
 *   direction w = (persistence*d - t*g) + randomness*(2u-1) with t = (1-persistence)/|g|, d = w/|w|;
 *   move by step_cells*d; leaving the grid ends the particle;
 *   height and gradient g from the bilinear patch through the four surrounding texel centres (indices
 *   clamped to the grid); the speed follows the Coulomb/Voellmy energy step
 *   v^2' = (v^2 + 2g(dz - mu*dl)) / (1 + 2g*ds/(xi*h)), dl = step_cells*cell_size, ds = sqrt(dl^2+dz^2);
 *   a non-positive numerator stops the particle where it is, as does the optional runout angle;
 *   at most step_limit steps.
 * counts: H*W uint32, the number of particle entries into each texel (the release texel counts once
 *   per particle). vmax: H*W float, the maximum speed (m/s) reached in each texel (0 if none).
 * stats (nullable): 4 uint64 on the device: {steps, particles that left the grid, that stopped, that
 *   reached step_limit}; "steps" counts every step entered, the terminating one included.
 * particles_per_cell >= 1; dem, mask, counts, vmax as above; H, W >= 1, both < 2^23; (H + 2) (W + 2) < 2^30
 * (the kernel reads a copy of the DEM with a one-texel border through 32-bit byte offsets);
 * workspace: avl_workspace_bytes(H, W) bytes of device memory, owned by the caller, not retained. */
AVL_API int avl_trajectories(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                     const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit, uint64_t seed,
                     uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                     size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): avl_trajectories without a workspace argument. The workspace lives in
 * a scratch array of avl_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on each GPU it runs
 * on until the process ends; the call allocates nothing, creates no HIP event and does not autotune (it
 * takes the variant an earlier avl_trajectories call tuned for a problem of this size, else variant 0;
 * results are the same for every variant). Arguments, results and errors are those of avl_trajectories,
 * plus AVL_EINVAL when avl_workspace_bytes(H, W) exceeds the scratch (about 1.6 M texels, e.g. 1280 x 1280)
 * and AVL_EHIP when the scratch's device address cannot be found. Every call on one GPU uses that GPU's
 * one scratch array, so calls that overlap on one GPU (other streams, other threads) race: serialise them.
 * Each call re-initialises what it reads from the scratch. */
AVL_API int avl_trajectories_noalloc(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                                     const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit,
                                     uint64_t seed, uint32_t run_id, uint32_t* counts, float* vmax, uint64_t* stats,
                                     void* stream);
AVL_API size_t avl_noalloc_scratch_bytes(void);

/* Debug paths (diagnostics: localising a difference from the model to one particle and one step, and the
 * real access pattern of a pass for the memory microbenchmarks): avl_trajectories with the paths of the
 * particles first .. first + n_rec - 1 recorded, particle k of the run being replica k % P of the k / P-th
 * release texel in row-major order. The pass runs the trajectory kernel's recording instantiation, whose
 * arithmetic is that of every other instantiation, so counts, vmax and stats are avl_trajectories' results.
 * ends (n_rec uint32, required): (accepted steps << 2) | end, end 0 = step limit, 1 = left the grid, 2 =
 *   stopped (energy line or runout angle); 0xFFFFFFFF for a k past the run's last particle.
 * points (nullable, float pairs (x, y) in cell units): point 0 is the release point, point m the position
 *   after the m-th accepted step, and a stopped particle's last point (m = steps + 1) the target of the
 *   step that stopped it. Particle k - first's point m goes to points[2 (offsets[k - first] + m)] when
 *   offsets (n_rec uint64) is given (the caller sizes each run of points from an earlier call's ends:
 *   steps + 1, plus 1 for a stop), else to points[2 ((k - first) stride + m)] for m < stride only.
 * speeds2 (nullable, needs points): v^2 at each point (0 at the release point and at a stop's target).
 * Other arguments, limits and errors as avl_trajectories; AVL_EINVAL also for n_rec = 0, no ends, or points
 * with neither offsets nor a stride >= 1. Every array is device memory. */
AVL_API int avl_trajectories_record(const float* dem, const uint8_t* mask, int32_t H, int32_t W, float cell_size,
                                    const avl_params* params, uint32_t particles_per_cell, uint32_t step_limit,
                                    uint64_t seed, uint32_t run_id, uint64_t first, uint32_t n_rec,
                                    const uint64_t* offsets, uint32_t stride, float* points, float* speeds2,
                                    uint32_t* ends, uint32_t* counts, float* vmax, uint64_t* stats, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* ---- Memory microbenchmarks (measurement: the ceilings of the trajectory node's memory traffic on this
 * chip, for a pass's own addresses). They take the output of avl_trajectories_record's two calls (ends, then
 * points and speeds2 at the offsets sized from the ends) over particles 0 .. n_particles - 1 of a run on an
 * H x W grid; the offsets must be those the points were written with. Nothing of the model is computed. With
 * avl_set_profiling on, avl_last_kernel_ms gives the replay kernel's duration.
 *
 * avl_bench_schedule lays the pass's memory operations out in the order a wave meets them: chunks of 64
 *   consecutive particles, and within a chunk the t-th operation of every particle that has one, in particle
 *   order. mode 0 writes per chunk c (of ceil(n_particles / 64)) totals[2c] = its gathers (each accepted step's
 *   position and a stopped particle's rejected target) and totals[2c + 1] = its cell visits (the release cell
 *   and every cell entered). mode 1 writes, at gather_base[c] and visit_base[c] (the exclusive sums of those
 *   totals), the gathers (u32 byte offset of the 2 x 2 patch in a copy of the DEM padded by one texel) and the
 *   visits (u32 pairs: the cell, the bits of the largest v^2 of the steps that ended in it). All device arrays.
 * avl_bench_gather: two 8-byte loads from the padded copy of dem (H*W floats) per gather, every gather
 *   independent; *checksum (device u32) gets the XOR of the bits of every texel read. workspace:
 *   avl_workspace_bytes(H, W).
 * avl_bench_atomics: per visit a device-scope u32 add to counts and a u32 max of the v^2 bits into vmax2_bits
 *   (H*W u32 each, overwritten): the accumulation without aggregation, whose rasters equal the pass's.
 * avl_bench_stream: copies `bytes` (a multiple of 16; 16-byte aligned pointers) from src to dst. */
AVL_API int avl_bench_schedule(int32_t mode, int32_t H, int32_t W, const float* points, const float* speeds2,
                               const uint64_t* offsets, const uint32_t* ends, uint64_t n_particles, uint64_t* totals,
                               const uint64_t* gather_base, const uint64_t* visit_base, uint32_t* gathers,
                               uint32_t* visits, void* stream);
AVL_API int avl_bench_gather(const float* dem, int32_t H, int32_t W, const uint32_t* gathers, uint64_t n_gathers,
                             uint32_t* checksum, void* workspace, size_t workspace_bytes, void* stream);
AVL_API int avl_bench_atomics(int32_t H, int32_t W, const uint32_t* visits, uint64_t n_visits, uint32_t* counts,
                              uint32_t* vmax2_bits, void* stream);
AVL_API int avl_bench_stream(const void* src, void* dst, size_t bytes, void* stream);

/* Release texture at a finer resolution than the DEM (section 5.2: the user picks the texture resolution
 * at which release points are evaluated; a known release area, as for the historic event of figure 1, can
 * be handed in as a texture of its own). The texture has mult x mult texels per DEM cell, row-major,
 * (mult*H) x (mult*W); texel (R, C) is centred at ((C + 1/2) / mult, (R + 1/2) / mult) in DEM cell units. */
#define AVL_MAX_RELEASE_MULT 16

/* Release map at mult texels per DEM cell edge: at each fine texel centre, nz (channel 2 of normals4) and
 * the height are filtered bilinearly between the DEM texel centres with clamped indices (the sample a
 * linear texture filter with clamp-to-edge addressing takes; nz is not renormalised), in binary32 as
 * top = a + fx(b - a), bottom = c + fx(d - c), value = top + fy(bottom - top), and tested as in
 * avl_release_mask. mult = 1 gives avl_release_mask's map. 1 <= mult <= AVL_MAX_RELEASE_MULT,
 * (mult H)(mult W) < 2^31, mult H and mult W < 2^23; mask: (mult*H)*(mult*W) bytes; other arguments as
 * avl_release_mask. */
AVL_API int avl_release_mask_fine(const float* normals4, const float* dem, int32_t H, int32_t W, int32_t mult,
                                  float slope_min_deg, float slope_max_deg, float z_min, float z_max, uint8_t* mask,
                                  void* stream);

/* Workspace bytes that avl_trajectories_fine needs (0 if an argument is out of range); mult = 1 gives
 * avl_workspace_bytes(H, W). */
AVL_API size_t avl_fine_workspace_bytes(int32_t H, int32_t W, int32_t mult);

/* avl_trajectories from a release texture with mult x mult texels per DEM cell (mask: (mult*H)*(mult*W)
 * bytes): particles_per_cell particles start at the centre of every nonzero texel, inside the DEM cell
 * (R / mult, C / mult), which counts their entry; their random stream has counter word 2 = the texel's
 * index R*(mult*W) + C in the texture. Rasters, stats and the model are those of avl_trajectories (DEM
 * resolution, H*W); mult = 1 is exactly avl_trajectories. 1 <= mult <= AVL_MAX_RELEASE_MULT,
 * (mult H)(mult W) < 2^31, mult H and mult W < 2^23 (release points are formed in binary32);
 * workspace: avl_fine_workspace_bytes(H, W, mult) bytes. */
AVL_API int avl_trajectories_fine(const float* dem, const uint8_t* mask, int32_t H, int32_t W, int32_t mult,
                                  float cell_size, const avl_params* params, uint32_t particles_per_cell,
                                  uint32_t step_limit, uint64_t seed, uint32_t run_id, uint32_t* counts, float* vmax,
                                  uint64_t* stats, void* workspace, size_t workspace_bytes, void* stream);

/* One run of a batch: which DEM tile, which release scenario (mask) and which parameter set, and the
 * run's random stream (Philox key = seed, counter word 3 = run_id). 24 bytes. */
typedef struct avl_run {
    uint32_t tile;     /* index into dems, < n_tiles */
    uint32_t scenario; /* index into masks, < n_masks */
    uint32_t param;    /* index into params, < n_params */
    uint32_t run_id;   /* Philox counter word 3 */
    uint64_t seed;     /* Philox key */
} avl_run;

/* Workspace bytes that avl_trajectories_batched needs (0 if a count is < 1): per mask, room for the
 * release-cell list and the particles' start states of every cell (36 bytes per DEM cell), plus a padded
 * copy of every tile and the run table. */
AVL_API size_t avl_batched_workspace_bytes(int32_t H, int32_t W, int32_t n_tiles, int32_t n_masks, int32_t n_runs);

/* Batched ensembles (section 5.2 motivates interactive sweeps of the trajectory parameters; section 3
 * recomputes the overlay whenever the user changes them): n_runs independent trajectory passes, each
 * exactly the avl_trajectories pass of its (tile, scenario, parameter set, seed, run_id), all in one
 * persistent launch over a shared particle queue.
 * dems: n_tiles*H*W floats (tile t at t*H*W). masks: n_masks*H*W bytes. params: n_params avl_params and
 * runs: n_runs avl_run, both DEVICE arrays (so a captured sequence can be replayed with new values).
 * counts, vmax: n_runs*H*W (run r at r*H*W), as in avl_trajectories. stats (nullable): n_runs*4 uint64.
 * run_status (nullable): n_runs int32, 0 = ran, 1 = an index out of range, 2 = invalid parameters (such a
 * run releases no particle and leaves zero rasters). particles_per_cell and step_limit are shared.
 * Need H, W < 2^23, n_runs*H*W, n_tiles*H*W, n_masks*H*W and n_tiles*(H+2)*(W+2) all < 2^32 - 1 and
 * (H+2)*(W+2) < 2^30 (the kernel reads padded copies of the tiles through 32-bit offsets). When `stream` is not the null stream, the
 * whole sequence (zero fills, compactions, run setup, trajectory kernel, finalize) is captured once into
 * a HIP graph per argument set and replayed on later calls. */
AVL_API int avl_trajectories_batched(const float* dems, int32_t n_tiles, const uint8_t* masks, int32_t n_masks,
                                     int32_t H, int32_t W, float cell_size, const avl_params* params,
                                     int32_t n_params, const avl_run* runs, int32_t n_runs,
                                     uint32_t particles_per_cell, uint32_t step_limit, uint32_t* counts, float* vmax,
                                     uint64_t* stats, int32_t* run_status, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* ---- Smooth variant and its adjoint (a differentiable runout field for calibrating mu, xi, h and the
 * release mass against a target deposit).
 * Every particle of release cell c carries mass[c] / particles_per_cell (mass NULL: 1 per cell). Paths
 * are those of avl_trajectories. A particle stopped by the energy step rests at the zero of that step's
 * energy numerator, the fraction t* = v^2 / (v^2 - num) of the step (0 when v^2 = 0); one stopped by the
 * runout angle or the step limit rests where it is; one that leaves the grid loses its mass. Its mass
 * is splatted bilinearly at the resting point (the height patch's four texel centres and weights,
 * clamped corners merging) into deposit_q, an H*W int64 raster in units of 2^-24 (order independent, so
 * bit-reproducible); deposit (nullable) gets it as float. With AVL_SMOOTH_VELOCITY every accepted step
 * also splats (mass per particle) * v at the new position into velocity_q / velocity.
 * max_release_cells: an upper bound on the number of release cells (it sizes the checkpoints); a mask with
 * more release cells releases nothing and sets *status = 3 (status: device int32, nullable).
 * stats as in avl_trajectories. H, W >= 1, both < 2^23, (H + 2)(W + 2) < 2^30 (as avl_trajectories; the same
 * limits hold for avl_trajectories_backward and avl_calibrate). workspace: avl_smooth_workspace_bytes(...) bytes;
 * it keeps the per-particle checkpoints (every 64 steps) that avl_trajectories_backward reads. */
#define AVL_SMOOTH_VELOCITY 1u
AVL_API size_t avl_smooth_workspace_bytes(int32_t H, int32_t W, int32_t max_release_cells,
                                          uint32_t particles_per_cell, uint32_t step_limit);
AVL_API int avl_trajectories_smooth(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                                    float cell_size, const avl_params* params, uint32_t particles_per_cell,
                                    uint32_t step_limit, uint64_t seed, uint32_t run_id, int32_t max_release_cells,
                                    uint32_t flags, int64_t* deposit_q, float* deposit, int64_t* velocity_q,
                                    float* velocity, uint64_t* stats, int32_t* status, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* Adjoint of the deposit of the preceding avl_trajectories_smooth call that used the same arguments and
 * workspace: given grad_deposit = dL/dD (H*W float), writes dparams = {dL/dmu, dL/dxi, dL/dh} (3 device
 * doubles) and dmass = dL/dmass (H*W float, 0 off the release cells). For each particle it recomputes the
 * last path segment from its checkpoint, takes dL/d(resting point) through the splat weights and the
 * fractional last step, then sweeps the v^2 recursion backward segment by segment, each segment
 * recomputed from its checkpoint. Sums run in binary64 in a fixed order (deterministic). per_particle
 * (nullable): 4 * max_release_cells * particles_per_cell floats, the per-particle dL/dmu, dL/dxi, dL/dh
 * and sum of gD * w, each block in release order. The velocity raster is not differentiated. */
AVL_API int avl_trajectories_backward(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                                      float cell_size, const avl_params* params, uint32_t particles_per_cell,
                                      uint32_t step_limit, uint64_t seed, uint32_t run_id, int32_t max_release_cells,
                                      const float* grad_deposit, double* dparams, float* dmass, float* per_particle,
                                      void* workspace, size_t workspace_bytes, void* stream);

/* ---- Calibration loop: Adam (Kingma and Ba, ICLR 2015, algorithm 1) on (mu, xi) against a target deposit,
 * the use the smooth variant and its adjoint exist for. Each iteration runs avl_trajectories_smooth at the
 * current (mu, xi) rounded to binary32, the loss L = sum (D - T)^2 / N over the H*W deposit D (the fixed
 * point raster as float) and its gradient dL/dD = c (D - T) with c = 2/N in binary32 (L summed in binary64
 * in a fixed order), then avl_trajectories_backward, and updates (mu, xi) in binary64 (on the device, one
 * thread, in this order of operations):
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;  theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * then clamps mu >= mu_min and xi >= xi_min. The other parameters stay those of *start. */
typedef struct avl_adam {
    float lr_mu, lr_xi;      /* step sizes, finite, > 0 (e.g. 0.003 and 30) */
    float beta1, beta2;      /* moment decay rates in [0, 1) (e.g. 0.9 and 0.999) */
    float eps;               /* denominator guard, finite, > 0 (e.g. 1e-8) */
    float mu_min, xi_min;    /* lower bounds of the iterates: finite, mu_min >= 0, xi_min > 0 */
} avl_adam;

/* Workspace bytes avl_calibrate needs (0 if an argument is out of range): the smooth pass's workspace plus
 * the deposit, its gradient, the reductions, the parameters, the optimiser state and 64 history rows. */
AVL_API size_t avl_calibrate_workspace_bytes(int32_t H, int32_t W, int32_t max_release_cells,
                                             uint32_t particles_per_cell, uint32_t step_limit);

/* n_iters Adam iterations from (start->mu, start->xi) (start->xi finite). target: H*W float deposit on the
 * device. history (host, nullable when n_iters = 0): n_iters rows of 5 doubles, (L, mu, xi, dL/dmu, dL/dxi)
 * at each iterate before its update. result (host): *start with the final mu and xi (binary32). The other
 * arguments are those of avl_trajectories_smooth. The parameters, the optimiser state and the rows stay on
 * the device: the host enqueues the iterations without waiting, the rows are copied back 64 at a time, and
 * the call waits for the stream once at the end. A mask with more release cells than max_release_cells, or
 * an iterate the run setup rejects, returns AVL_EINVAL after the loop (history then unspecified). */
AVL_API int avl_calibrate(const float* dem, const uint8_t* mask, const float* mass, int32_t H, int32_t W,
                          float cell_size, const avl_params* start, uint32_t particles_per_cell, uint32_t step_limit,
                          uint64_t seed, uint32_t run_id, int32_t max_release_cells, const float* target,
                          int32_t n_iters, const avl_adam* adam, double* history, avl_params* result,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Overlay mipmap (section 3: a mipmap of the full-resolution overlay texture is the multi-resolution
 * overlay the renderer samples). Level l + 1 halves level l, rounding up: its cell (r, c) covers cells
 * 2r..2r+1 x 2c..2c+1 of level l that exist. Entry counts add (uint64, so a coarse level cannot
 * overflow); speeds take the maximum. Levels 1 .. L-1 (L = avl_mipmap_levels(H, W), level 0 being the
 * input) are written one after the other, each row-major: counts_pyr and vmax_pyr hold
 * avl_mipmap_cells(H, W) entries (a grid of one cell has no coarser level and writes nothing).
 * counts (H*W uint32) and vmax (H*W float) as written by avl_trajectories; device pointers; H, W >= 1,
 * H*W < 2^31. Asynchronous on `stream`. */
AVL_API int32_t avl_mipmap_levels(int32_t H, int32_t W);
AVL_API int64_t avl_mipmap_cells(int32_t H, int32_t W);
AVL_API int avl_overlay_mipmap(const uint32_t* counts, const float* vmax, int32_t H, int32_t W, uint64_t* counts_pyr,
                               float* vmax_pyr, void* stream);

/* Tuning controls. variant: -1 = autotune (default: the first call per device and problem-size bucket
 * times every kernel variant and keeps the fastest; all variants give identical results), or a fixed
 * variant index in [0, avl_tuning_variants()). graphs: 1 = capture batched calls into HIP graphs
 * (default), 0 = launch eagerly. Returns AVL_EINVAL for an out-of-range variant. */
AVL_API int avl_set_tuning(int32_t variant, int32_t graphs);
AVL_API int32_t avl_tuning_variants(void);
/* The same for the smooth forward (avl_trajectories_smooth) and its adjoint (avl_trajectories_backward):
 * -1 lets the library's tuner pick a grid shape per problem size, else a fixed variant index in
 * [0, n) with n from avl_smooth_tuning_variants (grid shapes only: every variant gives identical
 * results). Returns AVL_EINVAL for an out-of-range index. */
AVL_API int avl_set_smooth_tuning(int32_t forward_variant, int32_t backward_variant);
/* Number of smooth forward and adjoint variants into *n_forward, *n_backward (host pointers); AVL_EINVAL
 * for a NULL pointer. */
AVL_API int avl_smooth_tuning_variants(int32_t* n_forward, int32_t* n_backward);
/* Shape of a kernel variant: info (8 host int32) = threads per block, iterations per epoch between table
 * flushes, LDS table slots per block, probes per key, window top-up in blocks of slots, retention threshold
 * (0 = none), waves per SIMD the register budget is sized for, particle slots per lane that size the grid of a
 * small problem. AVL_EINVAL for a NULL info or an index out of range. */
AVL_API int avl_tuning_variant_info(int32_t variant, int32_t* info);
/* The variant the last trajectory call on this thread used. */
AVL_API int32_t avl_last_variant(void);

/* Kernel timing (diagnostics; not for concurrent callers). With enable = 1, every later uncaptured
 * trajectory call (plain or batched) records a pair of HIP events on its stream around the trajectory
 * kernel alone; avl_last_kernel_ms waits for the last such pair and writes the kernel's duration in
 * milliseconds to *ms. Returns AVL_EINVAL if ms is NULL or no call was timed since profiling was
 * enabled, AVL_EHIP on a HIP error. enable = 0 stops the timing (the events are kept). */
AVL_API int avl_set_profiling(int32_t enable);
AVL_API int avl_last_kernel_ms(float* ms);

/* Tail probe (diagnostics; not for concurrent callers). With blocks3 set (a device buffer of 3 * n_blocks
 * uint64), every later uncaptured single-run trajectory call whose persistent grid has at most n_blocks blocks
 * writes, per block b, the GPU's 100 MHz real-time clock at the block's start (blocks3[3b]), when the block
 * first finds no particle slot left in its window or in any queue (3b + 1; 0 if it never does, i.e. if it left
 * at once) and at its end (3b + 2); the caller zeroes the buffer beforehand. blocks3 = NULL stops it.
 * avl_trajectory_grid gives the grid (blocks) of a kernel variant on the current device, -1 if out of range. */
AVL_API int avl_set_probe(uint64_t* blocks3, uint64_t n_blocks);
AVL_API int32_t avl_trajectory_grid(int32_t variant);

/* Name of an error code. Never NULL. */
AVL_API const char* avl_strerror(int code);

/* Detail of the last failed call on the calling thread ("" if none). Valid until the next call. */
AVL_API const char* avl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AVL_H */
