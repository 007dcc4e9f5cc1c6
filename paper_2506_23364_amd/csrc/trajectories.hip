// Particle trajectories of the avalanche overlay (section 5.2 of arXiv 2506.23364, the trajectory node):
// particles released per coded texel, steered by persistence and a random deviation from the optimal
// (downslope) path, slowed by Coulomb/Voellmy friction, stopped by the energy line or a runout angle;
// accumulated into a hit-count raster and a max-velocity raster.
//
// Design for gfx950 (measured choices; the alternatives are recorded in the design notes):
//  - One persistent grid sized to the chip's occupancy; one lane carries one particle at a time and its
//    whole state stays in VGPRs. A lane whose particle ended takes the next particle slot in the same
//    iteration, from a per-wave reservoir refilled 64 slots at a time from a device-wide counter.
//  - Slots are ordered replica-major within a release cell, so the 64 lanes of a wave mostly carry
//    replicas of one release cell: their 2x2 DEM gathers hit the same L2 lines, and their paths enter
//    the same cells.
//  - The slot range is split into one partition per XCD; a wave starts on its own XCD's partition and
//    moves on to the others only when it is empty. Each XCD's L2 then holds its own band of the DEM and
//    of the rasters instead of all eight caching the same band.
//  - Hit counts and per-cell max v^2 go first into a wave-private direct-mapped table in LDS (tag,
//    count, max), flushed to the rasters every kFlushEvery iterations. Replicas on overlapping paths
//    then cost one global atomic per cell and flush period instead of one per entry. A cell whose slot
//    is held by another cell goes straight to the global raster.
//  - The global rasters are private per XCD (merged after the kernel), so no two XCDs update one line.
//  - Accumulation is integer only (u32 add; u32 max on the bits of v^2 >= 0, whose order is the value
//    order), so every raster is independent of scheduling: bit-reproducible.
//  - Philox4x32-10 gives four words per block; one block serves two consecutive steps.
#include "avl_internal.h"

namespace avl {

namespace {

constexpr int kTbl = 256;          // table slots per wave (power of two)
constexpr int kFlushEvery = 16;    // iterations between table flushes
constexpr uint32_t kChunk = 64;    // particle slots taken from a queue per reservoir refill
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 multiply-xor bijection with a Weyl key
// schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// 24 random bits -> uniform in [-1, 1), exact in binary32
__device__ __forceinline__ float signed_unit(uint32_t u) {
    return 2.0f * ((float)(u >> 8) * 5.9604644775390625e-8f) - 1.0f;
}

struct Sample {
    float z, gx, gy;
};

// Bilinear patch through the four texel centres around (x, y), indices clamped to the grid.
__device__ __forceinline__ Sample bilinear(const float* __restrict__ dem, int H, int W, float x, float y) {
    const float sx = x - 0.5f, sy = y - 0.5f;
    const float fc = floorf(sx), fr = floorf(sy);
    const float fx = sx - fc, fy = sy - fr;
    const int c0 = (int)fc, r0 = (int)fr;
    const int ca = min(max(c0, 0), W - 1), cb = min(max(c0 + 1, 0), W - 1);
    const int ra = min(max(r0, 0), H - 1), rb = min(max(r0 + 1, 0), H - 1);
    const float* rowa = dem + (size_t)ra * W;
    const float* rowb = dem + (size_t)rb * W;
    const float a = rowa[ca], b = rowa[cb], c = rowb[ca], d = rowb[cb];
    const float top = a + fx * (b - a);
    const float bot = c + fx * (d - c);
    Sample s;
    s.z = top + fy * (bot - top);
    s.gx = (b - a) + fy * ((d - c) - (b - a));
    s.gy = bot - top;
    return s;
}

__device__ __forceinline__ uint64_t wave_bcast64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint32_t xcd_id() {
    // HW_REG_XCC_ID bits [3:0]: the XCD this wave runs on
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (uint32_t)(kXcds - 1);
}

__device__ __forceinline__ uint32_t slot_of(uint32_t key) {
    return (key * 0x9E3779B1u) >> (32 - 8);  // kTbl = 2^8
}
static_assert(kTbl == 256, "slot_of assumes 256 slots");

// LDS table accesses are relaxed atomics: lanes of the wave update slots concurrently.
__device__ __forceinline__ uint32_t lds_ld(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Max into a global raster cell. v^2 only grows, so a stale read that is already >= v proves the
// atomic unnecessary.
__device__ __forceinline__ void global_max(uint32_t* __restrict__ p, uint32_t bits) {
    if (__builtin_nontemporal_load(p) < bits) atomicMax(p, bits);
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_trajectories(TrajArgs a) {
    __shared__ uint32_t s_tag[kWavesPerBlock][kTbl], s_cnt[kWavesPerBlock][kTbl], s_vmx[kWavesPerBlock][kTbl];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    uint32_t* const tag = s_tag[wv];
    uint32_t* const cnt = s_cnt[wv];
    uint32_t* const vmx = s_vmx[wv];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint64_t total = (uint64_t)(uint32_t)(*a.n_cells) * (uint64_t)a.P;
    const int W = a.W, H = a.H;
    const float fW = (float)W, fH = (float)H;
    const uint32_t xcd = xcd_id();
    const size_t n_cells_grid = (size_t)H * W;
    uint32_t* const counts = a.counts + xcd * n_cells_grid;
    uint32_t* const vmax2 = a.vmax2 + xcd * n_cells_grid;

    for (int k = lane; k < kTbl; k += kWave) {
        lds_st(tag + k, kEmpty);
        lds_st(cnt + k, 0u);
        lds_st(vmx + k, 0u);
    }

    // table slot of `key`, claimed if empty; -1 if the slot belongs to another cell
    auto claim = [&](uint32_t key) -> int {
        const uint32_t sl = slot_of(key);
        uint32_t t = lds_ld(tag + sl);
        if (t == kEmpty) {
            const uint32_t old = atomicCAS(tag + sl, kEmpty, key);
            t = (old == kEmpty) ? key : old;
        }
        return t == key ? (int)sl : -1;
    };
    auto flush = [&]() {
        for (int k = lane; k < kTbl; k += kWave) {
            const uint32_t t = lds_ld(tag + k);
            if (t != kEmpty) {
                const uint32_t c = lds_ld(cnt + k), v = lds_ld(vmx + k);
                if (c) atomicAdd(counts + t, c);
                if (v) global_max(vmax2 + t, v);
                lds_st(cnt + k, 0u);
                lds_st(vmx + k, 0u);
                lds_st(tag + k, kEmpty);
            }
        }
    };

    // wave-uniform queue state: partition being drained, partitions found empty, slot reservoir
    uint32_t part = xcd;
    uint32_t tried = 0;
    bool queue_empty = (total == 0);
    uint64_t res_next = 0, res_end = 0;

    // lane state
    bool alive = false;
    float x = 0, y = 0, z = 0, gx = 0, gy = 0, dx = 0, dy = 0, v2 = 0, x0 = 0, y0 = 0, zr = 0, cmax2 = 0;
    uint32_t n = 0, rep = 0, cell_id = 0, spare_x = 0, spare_y = 0, cur = 0;
    int my_slot = -1;  // table slot of the current cell, -1 if none
    uint64_t lane_steps = 0;
    uint32_t n_exit = 0, n_stop = 0, n_limit = 0;

    for (uint32_t iter = 1;; ++iter) {
        const uint64_t idle = __ballot(!alive);
        const int nidle = __popcll(idle);
        const bool drained = queue_empty && res_next >= res_end;
        if (nidle == kWave && drained) break;
        if (iter % kFlushEvery == 0) {
            flush();
            my_slot = -1;
        }

        // ---- hand slots to idle lanes in lane order: reservoir first, then a new chunk
        bool fresh = false;
        if (nidle > 0 && !drained) {
            const uint64_t avail = res_end - res_next;
            const int rank = __popcll(idle & below);
            uint64_t slot = ~0ull;
            if (avail >= (uint64_t)nidle) {
                slot = res_next + rank;
                res_next += nidle;
            } else {
                uint64_t base = 0, cend = 0;
                const int leader = __ffsll((long long)idle) - 1;
                while (!queue_empty) {
                    const uint64_t pb = total * part / kXcds, pe = total * (part + 1) / kXcds;
                    uint64_t got = 0;
                    if (lane == leader) got = atomicAdd(a.queues + part, (unsigned long long)kChunk);
                    got = wave_bcast64(__shfl(got, leader, kWave));
                    if (pb + got < pe) {
                        base = pb + got;
                        cend = (base + kChunk < pe) ? base + kChunk : pe;
                        break;
                    }
                    part = (part + 1) % kXcds;
                    if (++tried >= (uint32_t)kXcds) queue_empty = true;
                }
                if ((uint64_t)rank < avail)
                    slot = res_next + rank;
                else if (base + (rank - avail) < cend)
                    slot = base + (rank - avail);
                const uint64_t next = base + ((uint64_t)nidle - avail);
                res_next = next < cend ? next : cend;
                res_end = cend;
            }
            if (!alive && slot < total) {
                // release particle `slot`: cell list entry slot / P, replica slot % P
                const uint64_t i = slot / a.P;
                rep = (uint32_t)(slot - i * a.P);
                cell_id = (uint32_t)a.cells[i];
                const int r = (int)(cell_id / (uint32_t)W);
                const int c = (int)(cell_id - (uint32_t)r * (uint32_t)W);
                x = (float)c + 0.5f;
                y = (float)r + 0.5f;
                const Sample s0 = bilinear(a.dem, H, W, x, y);
                z = s0.z;
                gx = s0.gx;
                gy = s0.gy;
                x0 = x;
                y0 = y;
                zr = z;
                const float gg = gx * gx + gy * gy;
                if (gg > 0.0f) {
                    const float t = 1.0f / sqrtf(gg);
                    dx = -(gx * t);
                    dy = -(gy * t);
                } else {
                    dx = 0.0f;
                    dy = 0.0f;
                }
                v2 = 0.0f;
                cmax2 = 0.0f;
                n = 0;
                cur = cell_id;
                alive = true;
                fresh = true;
            }
        }
        if (fresh) {  // entry into the release cell
            my_slot = claim(cur);
            if (my_slot >= 0)
                atomicAdd(cnt + my_slot, 1u);
            else
                atomicAdd(counts + cur, 1u);
        }

        // ---- one step of every live particle
        bool leave = false, entered = false;
        uint32_t leave_bits = 0;
        int leave_slot = -1;
        uint32_t leave_key = 0;
        if (alive) {
            bool ended = false;
            if (n >= a.S) {
                ++n_limit;
                ended = true;
            } else {
                ++lane_steps;
                uint32_t ux, uy;
                if ((n & 1u) == 0u) {
                    const uint4 o = philox4x32_10(n >> 1, rep, cell_id, a.run, a.key0, a.key1);
                    ux = o.x;
                    uy = o.y;
                    spare_x = o.z;
                    spare_y = o.w;
                } else {
                    ux = spare_x;
                    uy = spare_y;
                }
                const float rx = signed_unit(ux), ry = signed_unit(uy);
                const float gg = gx * gx + gy * gy;
                const float t = gg > 0.0f ? a.Q / sqrtf(gg) : 0.0f;
                const float wx = (a.per * dx - t * gx) + a.rnd * rx;
                const float wy = (a.per * dy - t * gy) + a.rnd * ry;
                const float ww = wx * wx + wy * wy;
                if (ww > 0.0f) {
                    const float inv = 1.0f / sqrtf(ww);
                    dx = wx * inv;
                    dy = wy * inv;
                }
                const float x1 = x + a.L * dx;
                const float y1 = y + a.L * dy;
                const float fc1 = floorf(x1), fr1 = floorf(y1);
                if (!(fc1 >= 0.0f && fc1 < fW && fr1 >= 0.0f && fr1 < fH)) {
                    ++n_exit;
                    ended = true;
                } else {
                    const Sample s1 = bilinear(a.dem, H, W, x1, y1);
                    const float dz = z - s1.z;
                    const float ds = sqrtf(a.dl2 + dz * dz);
                    const float num = v2 + a.g2 * (dz - a.mdl);
                    bool stop = !(num > 0.0f);
                    float v2n = 0.0f;
                    if (!stop) {
                        v2n = num / (1.0f + a.cd * ds);
                        if (a.use_alpha) {
                            const float hx = x1 - x0, hy = y1 - y0;
                            stop = (zr - s1.z) < a.tca * sqrtf(hx * hx + hy * hy);
                        }
                    }
                    if (stop) {
                        ++n_stop;
                        ended = true;
                    } else {
                        x = x1;
                        y = y1;
                        z = s1.z;
                        gx = s1.gx;
                        gy = s1.gy;
                        v2 = v2n;
                        ++n;
                        const uint32_t nc = (uint32_t)(int)fr1 * (uint32_t)W + (uint32_t)(int)fc1;
                        if (nc != cur) {
                            leave = cmax2 > 0.0f;
                            leave_bits = __float_as_uint(cmax2);
                            leave_slot = my_slot;
                            leave_key = cur;
                            cur = nc;
                            cmax2 = v2;
                            entered = true;
                        } else if (v2 > cmax2) {
                            cmax2 = v2;
                        }
                    }
                }
            }
            if (ended) {
                leave = cmax2 > 0.0f;
                leave_bits = __float_as_uint(cmax2);
                leave_slot = my_slot;
                leave_key = cur;
                alive = false;
            }
        }
        // ---- accumulate: max of the cell left, entry count of the cell entered
        if (leave) {
            int sl = leave_slot;
            if (sl < 0) sl = claim(leave_key);
            if (sl >= 0)
                atomicMax(vmx + sl, leave_bits);
            else
                global_max(vmax2 + leave_key, leave_bits);
        }
        if (entered) {
            my_slot = claim(cur);
            if (my_slot >= 0)
                atomicAdd(cnt + my_slot, 1u);
            else
                atomicAdd(counts + cur, 1u);
        }
    }
    flush();

    // per-wave totals
    const uint64_t s_steps = wave_sum64(lane_steps);
    const uint64_t s_exit = wave_sum64(n_exit), s_stop = wave_sum64(n_stop), s_limit = wave_sum64(n_limit);
    if (lane == 0) {
        if (s_steps) atomicAdd(a.stats + 0, (unsigned long long)s_steps);
        if (s_exit) atomicAdd(a.stats + 1, (unsigned long long)s_exit);
        if (s_stop) atomicAdd(a.stats + 2, (unsigned long long)s_stop);
        if (s_limit) atomicAdd(a.stats + 3, (unsigned long long)s_limit);
    }
}

hipError_t launch_trajectories(const TrajArgs& a, const LaunchShape& shape, hipStream_t s) {
    hipLaunchKernelGGL(k_trajectories, dim3(shape.grid), dim3(shape.block), 0, s, a);
    return hipGetLastError();
}

LaunchShape trajectory_shape() {
    int dev = 0;
    LaunchShape sh{kBlock, 2048};
    if (hipGetDevice(&dev) != hipSuccess) return sh;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return sh;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_trajectories),
                                                     sh.block, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 4;
    sh.grid = cus * per_cu;
    return sh;
}

}  // namespace avl
