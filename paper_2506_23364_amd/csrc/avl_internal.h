// Internal declarations shared by the libavl translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace avl {

constexpr int kWave = 64;

// ------------------------------------------------------------------ workspace layout
// [0, 256)            control block: n_cells (i32 @0), internal stats (4 x u64 @16), one particle-slot
//                     queue per XCD (kXcds x u64 @64)
// [256, 256 + B)      per-block counts / offsets of the compaction scan (u32 each), B rounded to 256
// [.., .. + 4 H W)    release-cell list (i32), rounded to 256
// [.., .. + 2 kXcds 4 H W)  per-XCD private count rasters, then per-XCD private v^2-bit rasters
constexpr int kXcds = 8;            // MI355X: 8 XCDs, each with its own L2
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanChunk = kScanThreads * kScanPerThread;  // cells per compaction block

inline size_t round256(size_t v) { return (v + 255) & ~size_t(255); }
inline int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

struct Workspace {
    int32_t* n_cells;
    unsigned long long* queues;  // kXcds counters
    unsigned long long* stats;
    uint32_t* blk;
    int32_t* cells;
    uint32_t* priv_counts;  // kXcds x H*W
    uint32_t* priv_vmax2;   // kXcds x H*W
};

size_t workspace_bytes(int64_t n);
Workspace carve(void* base, int64_t n);

// ------------------------------------------------------------------ trajectory kernel arguments
struct TrajArgs {
    const float* __restrict__ dem;
    const int32_t* __restrict__ cells;
    const int32_t* __restrict__ n_cells;
    unsigned long long* __restrict__ queues;  // kXcds slot counters, zero at launch
    uint32_t* __restrict__ counts;  // kXcds private count rasters (H*W each), zero at launch
    uint32_t* __restrict__ vmax2;   // kXcds private rasters of the binary32 bits of the per-cell max of v^2
                                    // (v^2 >= 0, so bit order is value order), zero at launch
    unsigned long long* __restrict__ stats;
    int32_t H, W;
    float g2, per, Q, rnd, L, dl2, mdl, cd, tca;
    int32_t use_alpha;
    uint32_t P, S, run, key0, key1;
};

struct LaunchShape {
    int block;  // threads per block (multiple of 64)
    int grid;   // blocks
};

// ------------------------------------------------------------------ launchers (enqueue only; return hipError_t)
hipError_t launch_normals(const float* dem, int H, int W, float cs, float* out4, hipStream_t s);
hipError_t launch_release_mask(const float* normals4, const float* dem, int64_t n, float cmin, float cmax,
                               float zmin, float zmax, uint8_t* mask, hipStream_t s);
hipError_t launch_compact(const uint8_t* mask, int64_t n, int32_t* cells, int32_t* n_cells, uint32_t* blk,
                          hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);
hipError_t launch_merge_rasters(const uint32_t* priv_counts, const uint32_t* priv_vmax2, int64_t n, uint32_t* counts,
                                float* vmax, hipStream_t s);
hipError_t launch_trajectories(const TrajArgs& a, const LaunchShape& shape, hipStream_t s);

// persistent-grid shape for the trajectory kernel on the current device
LaunchShape trajectory_shape();

}  // namespace avl
