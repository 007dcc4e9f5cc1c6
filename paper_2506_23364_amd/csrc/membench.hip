// Memory microbenchmarks that bound the trajectory pass (section 5.2, the trajectory node): they replay the
// memory operations of a recorded pass (avl_trajectories_record) without its arithmetic, so their rates are
// the ceilings of the pass's gathers and of its raster atomics on this chip, for the pass's own access
// stream.
//  - Gather replay: every 2 x 2 patch read of the pass (each accepted step's target and a stopped particle's
//    rejected target), as the pass reads it: two 8-byte loads from the padded DEM through a buffer
//    resource. Lanes take particles in slot order from per-XCD queues, 64 consecutive slots per wave, as
//    the pass does, so a wave's lanes walk neighbouring paths together.
//  - Atomic replay: the accumulation of the model without any aggregation: one device-scope u32 add per
//    cell entry and one u32 max of v^2 bits per cell left (the in-register cell maximum), straight to the
//    rasters. Its counts and maxima equal the pass's.
//  - HBM stream: a 16-byte-per-lane copy.
#include "particle.h"

namespace avl {

using namespace dev;

namespace {

constexpr int kReplayBlock = 256;

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v ^= (uint32_t)__shfl_xor((int)v, d, kWave);
    return v;
}

struct ReplayLane {
    bool alive = false;
    uint64_t at = 0;     // index of the lane's next point
    uint32_t left = 0;   // points left
};

}  // namespace

// Gather replay: the XOR of the bits of every texel read goes to *checksum (order-independent, so a host
// check can recompute it).
__global__ __launch_bounds__(kReplayBlock) void k_replay_gather(const float2* __restrict__ pts,
                                                               const unsigned long long* __restrict__ off,
                                                               const uint32_t* __restrict__ ends, uint64_t n,
                                                               const float* __restrict__ dem_pad, uint32_t pad_bytes,
                                                               int W, unsigned long long* __restrict__ queues,
                                                               uint32_t* __restrict__ checksum) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(dem_pad, pad_bytes);
    const uint32_t Wp = (uint32_t)W + 2u, row_bytes = 4u * Wp;
    Dispenser disp;
    disp.init(n, xcd_id());
    ReplayLane L;
    uint32_t acc = 0;
    for (;;) {
        const uint64_t idle = __ballot(!L.alive);
        if (__popcll(idle) == kWave && disp.drained()) break;
        if (idle && !disp.drained()) {
            const uint64_t slot = disp.take(queues, idle, lane, below);
            if (!L.alive && slot < n) {
                const uint32_t e = ends[slot];
                const uint32_t gathers = (e >> 2) + ((e & 3u) == 2u ? 1u : 0u);
                if (e != ~0u && gathers > 0u) {
                    L.alive = true;
                    L.at = off[slot] + 1;  // point 0 is the release point, read from the start records
                    L.left = gathers;
                }
            }
        }
        if (!L.alive) continue;
        const float2 p = pts[L.at];
        const float sx = p.x - 0.5f, sy = p.y - 0.5f;
        const uint32_t o = (__umul24((uint32_t)((int)floorf(sy) + 1), Wp) + (uint32_t)((int)floorf(sx) + 1)) * 4u;
        const auto ab = __builtin_amdgcn_raw_buffer_load_b64(rs, o, 0, 0);
        const auto cd = __builtin_amdgcn_raw_buffer_load_b64(rs, o, row_bytes, 0);
        acc ^= ab[0] ^ ab[1] ^ cd[0] ^ cd[1];
        ++L.at;
        if (--L.left == 0u) L.alive = false;
    }
    acc = wave_xor(acc);
    if (lane == 0 && acc) atomicXor(checksum, acc);
}

// Atomic replay: counts and the bits of the per-cell max of v^2, as the pass accumulates them but with no
// aggregation (every entry and every cell exit is a device-scope atomic).
__global__ __launch_bounds__(kReplayBlock) void k_replay_atomics(const float2* __restrict__ pts,
                                                                const float* __restrict__ v2s,
                                                                const unsigned long long* __restrict__ off,
                                                                const uint32_t* __restrict__ ends, uint64_t n, int W,
                                                                unsigned long long* __restrict__ queues,
                                                                uint32_t* __restrict__ counts,
                                                                uint32_t* __restrict__ vmax2) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    Dispenser disp;
    disp.init(n, xcd_id());
    ReplayLane L;
    uint32_t cur = 0;
    float cmax = 0.0f;
    for (;;) {
        const uint64_t idle = __ballot(!L.alive);
        if (__popcll(idle) == kWave && disp.drained()) break;
        if (idle && !disp.drained()) {
            const uint64_t slot = disp.take(queues, idle, lane, below);
            if (!L.alive && slot < n) {
                const uint32_t e = ends[slot];
                if (e != ~0u) {
                    const float2 p = pts[off[slot]];
                    cur = (uint32_t)(int)floorf(p.y) * (uint32_t)W + (uint32_t)(int)floorf(p.x);
                    atomicAdd(counts + cur, 1u);  // entry into the release cell
                    cmax = 0.0f;
                    L.alive = (e >> 2) > 0u;
                    L.at = off[slot] + 1;
                    L.left = e >> 2;
                }
            }
        }
        if (!L.alive) continue;
        const float2 p = pts[L.at];
        const float v2 = v2s[L.at];
        const uint32_t cell = (uint32_t)(int)floorf(p.y) * (uint32_t)W + (uint32_t)(int)floorf(p.x);
        if (cell != cur) {
            if (cmax > 0.0f) atomicMax(vmax2 + cur, __float_as_uint(cmax));
            atomicAdd(counts + cell, 1u);
            cur = cell;
            cmax = v2;
        } else if (v2 > cmax) {
            cmax = v2;
        }
        ++L.at;
        if (--L.left == 0u) {
            L.alive = false;
            if (cmax > 0.0f) atomicMax(vmax2 + cur, __float_as_uint(cmax));
        }
    }
}

__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

namespace {

int replay_grid(const void* kernel) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kReplayBlock, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return cus * per_cu;
}

}  // namespace

hipError_t launch_replay_gather(const float2* pts, const unsigned long long* off, const uint32_t* ends, uint64_t n,
                                const float* dem_pad, uint32_t pad_bytes, int W, unsigned long long* queues,
                                uint32_t* checksum, hipStream_t s) {
    hipLaunchKernelGGL(k_replay_gather, dim3(replay_grid(reinterpret_cast<const void*>(&k_replay_gather))),
                       dim3(kReplayBlock), 0, s, pts, off, ends, n, dem_pad, pad_bytes, W, queues, checksum);
    return hipGetLastError();
}

hipError_t launch_replay_atomics(const float2* pts, const float* v2s, const unsigned long long* off,
                                 const uint32_t* ends, uint64_t n, int W, unsigned long long* queues, uint32_t* counts,
                                 uint32_t* vmax2, hipStream_t s) {
    hipLaunchKernelGGL(k_replay_atomics, dim3(replay_grid(reinterpret_cast<const void*>(&k_replay_atomics))),
                       dim3(kReplayBlock), 0, s, pts, v2s, off, ends, n, W, queues, counts, vmax2);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, uint64_t n16, hipStream_t s) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    uint64_t blocks = (n16 + 255) / 256;
    const uint64_t cap = (uint64_t)cus * 16;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace avl
