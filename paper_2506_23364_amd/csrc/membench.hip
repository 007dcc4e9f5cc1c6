// Memory microbenchmarks that bound the trajectory pass (section 5.2, the trajectory node): they replay the
// memory operations of a recorded pass (avl_trajectories_record) without its arithmetic and without its
// dependences, so their rates are the ceilings of the pass's gathers and of its raster atomics on this chip,
// for the pass's own addresses.
//
// A schedule kernel first lays the pass's operations out in the order a wave meets them: particles in
// chunks of 64 consecutive slots (the pass's unit of work: replicas of neighbouring release texels), and
// within a chunk step by step, the t-th operation of every particle of the chunk that has one, in lane
// order. The replays then stream that schedule with every operation independent of the others:
//  - gathers: each entry is the byte offset of a 2 x 2 patch in the padded DEM (every accepted step's
//    position and a stopped particle's rejected target); the replay issues two 8-byte buffer loads per entry,
//    as the pass does.
//  - atomics: each entry is one cell visit (the cell and the largest v^2 of the steps that ended in it); the
//    replay issues a device-scope u32 add (the entry) and a u32 max of the v^2 bits, the accumulation of the
//    model with no aggregation. Its rasters equal the pass's.
//  - HBM stream: a copy, four 16-byte loads in flight per lane.
#include "particle.h"

namespace avl {

using namespace dev;

namespace {

constexpr int kSchedBlock = 256;  // four chunks (waves) per block
constexpr int kReplayBlock = 256;
constexpr int kUnroll = 4;        // independent operations in flight per lane

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v ^= (uint32_t)__shfl_xor((int)v, d, kWave);
    return v;
}

__device__ __forceinline__ uint32_t cell_of(float2 p, int W) {
    return (uint32_t)(int)floorf(p.y) * (uint32_t)W + (uint32_t)(int)floorf(p.x);
}

}  // namespace

// One wave per chunk of 64 particles. mode 0: per chunk, the number of gathers and of cell visits (into
// totals[2 c], totals[2 c + 1]); mode 1: the chunk's entries at the bases (exclusive scans of the totals).
__global__ __launch_bounds__(kSchedBlock) void k_replay_schedule(int mode, const float2* __restrict__ pts,
                                                                 const float* __restrict__ v2s,
                                                                 const unsigned long long* __restrict__ off,
                                                                 const uint32_t* __restrict__ ends, uint64_t n, int W,
                                                                 unsigned long long* __restrict__ totals,
                                                                 const unsigned long long* __restrict__ gbase,
                                                                 const unsigned long long* __restrict__ vbase,
                                                                 uint32_t* __restrict__ gathers,
                                                                 uint2* __restrict__ visits) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint64_t n_chunks = (n + kWave - 1) / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * (kSchedBlock / kWave);
    const uint32_t Wp = (uint32_t)W + 2u;
    for (uint64_t c = (uint64_t)blockIdx.x * (kSchedBlock / kWave) + threadIdx.x / kWave; c < n_chunks; c += waves) {
        const uint64_t k = c * kWave + (uint64_t)lane;
        uint32_t e = ~0u;
        if (k < n) e = ends[k];
        const bool valid = e != ~0u;
        const uint32_t steps = valid ? e >> 2 : 0u;
        const uint32_t ng = valid ? steps + ((e & 3u) == 2u ? 1u : 0u) : 0u;
        const uint64_t o = valid ? off[k] : 0ull;
        // gathers: the t-th of every particle that has one, lane order
        uint64_t gat = mode ? gbase[c] : 0ull;
        for (uint32_t t = 0;; ++t) {
            const bool act = t < ng;
            const uint64_t m = __ballot(act);
            if (m == 0ull) break;
            if (mode && act) {
                const float2 p = pts[o + 1 + t];
                const uint32_t fr = (uint32_t)((int)floorf(p.y - 0.5f) + 1), fc = (uint32_t)((int)floorf(p.x - 0.5f) + 1);
                gathers[gat + (uint64_t)__popcll(m & below)] = (fr * Wp + fc) * 4u;
            }
            gat += (uint64_t)__popcll(m);
        }
        // visits: the release cell, then every cell entered; each with the largest v^2 of its steps
        uint64_t vat = mode ? vbase[c] : 0ull;
        uint32_t at = 0;  // next point to walk (point 0 is the release point)
        for (;;) {
            const bool act = valid && at <= steps;
            const uint64_t m = __ballot(act);
            if (m == 0ull) break;
            uint32_t cell = 0, bits = 0;
            if (act) {
                cell = cell_of(pts[o + at], W);
                float cmax = at == 0 ? 0.0f : v2s[o + at];
                ++at;
                while (at <= steps) {  // the visit goes on while the steps end in the same cell
                    const float2 p = pts[o + at];
                    if (cell_of(p, W) != cell) break;
                    const float v = v2s[o + at];
                    cmax = v > cmax ? v : cmax;
                    ++at;
                }
                bits = __float_as_uint(cmax);
            }
            if (mode && act) visits[vat + (uint64_t)__popcll(m & below)] = make_uint2(cell, bits);
            vat += (uint64_t)__popcll(m);
        }
        if (!mode && lane == 0) {
            totals[2 * c] = gat;
            totals[2 * c + 1] = vat;
        }
    }
}

// Gather replay: two 8-byte loads per schedule entry, kUnroll entries in flight per lane; the XOR of the bits
// of every texel read goes to *checksum (order-independent, so the host can check it).
__global__ __launch_bounds__(kReplayBlock) void k_replay_gather(const uint32_t* __restrict__ sched, uint64_t n,
                                                               const float* __restrict__ dem_pad, uint32_t pad_bytes,
                                                               uint32_t row_bytes, uint32_t* __restrict__ checksum) {
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(dem_pad, pad_bytes);
    const uint64_t T = (uint64_t)gridDim.x * kReplayBlock;
    uint32_t acc = 0;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kReplayBlock + threadIdx.x; i0 < n; i0 += T * kUnroll) {
        uint32_t o[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * T;
            o[u] = i < n ? sched[i] : ~0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (o[u] == ~0u) continue;
            const auto ab = __builtin_amdgcn_raw_buffer_load_b64(rs, o[u], 0, 0);
            const auto cd = __builtin_amdgcn_raw_buffer_load_b64(rs, o[u], row_bytes, 0);
            acc ^= ab[0] ^ ab[1] ^ cd[0] ^ cd[1];
        }
    }
    acc = wave_xor(acc);
    if ((threadIdx.x & (kWave - 1)) == 0 && acc) atomicXor(checksum, acc);
}

// Atomic replay: per schedule entry a u32 add of one entry and a u32 max of the visit's v^2 bits.
__global__ __launch_bounds__(kReplayBlock) void k_replay_atomics(const uint2* __restrict__ sched, uint64_t n,
                                                                uint32_t* __restrict__ counts,
                                                                uint32_t* __restrict__ vmax2) {
    const uint64_t T = (uint64_t)gridDim.x * kReplayBlock;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kReplayBlock + threadIdx.x; i0 < n; i0 += T * kUnroll) {
        uint2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * T;
            v[u] = i < n ? sched[i] : make_uint2(~0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (v[u].x == ~0u) continue;
            atomicAdd(counts + v[u].x, 1u);
            if (v[u].y) atomicMax(vmax2 + v[u].x, v[u].y);
        }
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     uint64_t n) {
    const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += T * kUnroll) {
        u32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * T;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * T;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

namespace {

int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

unsigned stream_blocks(uint64_t items, int threads) {
    const uint64_t want = (items + (uint64_t)threads * kUnroll - 1) / ((uint64_t)threads * kUnroll);
    const uint64_t cap = (uint64_t)device_cus() * 8;  // eight blocks of 256 per CU: 32 waves, full occupancy
    return (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

hipError_t launch_replay_schedule(int mode, const float2* pts, const float* v2s, const unsigned long long* off,
                                  const uint32_t* ends, uint64_t n, int W, unsigned long long* totals,
                                  const unsigned long long* gbase, const unsigned long long* vbase, uint32_t* gathers,
                                  uint2* visits, hipStream_t s) {
    const uint64_t chunks = (n + kWave - 1) / kWave;
    const uint64_t blocks = (chunks + (kSchedBlock / kWave) - 1) / (kSchedBlock / kWave);
    const uint64_t cap = (uint64_t)device_cus() * 8;
    const unsigned g = (unsigned)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
    hipLaunchKernelGGL(k_replay_schedule, dim3(g), dim3(kSchedBlock), 0, s, mode, pts, v2s, off, ends, n, W, totals,
                       gbase, vbase, gathers, visits);
    return hipGetLastError();
}

hipError_t launch_replay_gather(const uint32_t* sched, uint64_t n, const float* dem_pad, uint32_t pad_bytes,
                                uint32_t row_bytes, uint32_t* checksum, hipStream_t s) {
    hipLaunchKernelGGL(k_replay_gather, dim3(stream_blocks(n, kReplayBlock)), dim3(kReplayBlock), 0, s, sched, n,
                       dem_pad, pad_bytes, row_bytes, checksum);
    return hipGetLastError();
}

hipError_t launch_replay_atomics(const uint2* sched, uint64_t n, uint32_t* counts, uint32_t* vmax2, hipStream_t s) {
    hipLaunchKernelGGL(k_replay_atomics, dim3(stream_blocks(n, kReplayBlock)), dim3(kReplayBlock), 0, s, sched, n,
                       counts, vmax2);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, uint64_t n16, hipStream_t s) {
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3(stream_blocks(n16, 256)), dim3(256), 0, s, static_cast<const u32x4*>(src),
                       static_cast<u32x4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace avl
