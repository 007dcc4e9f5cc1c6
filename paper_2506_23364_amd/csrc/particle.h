// Device helpers shared by the particle kernels (plain, batched, smooth forward and adjoint): the
// random stream, the bilinear height patch and the wave-level queue utilities. Internal header.
#pragma once

#include "avl_internal.h"

namespace avl {
namespace dev {

constexpr uint32_t kChunk = 64;  // particle slots taken from a queue per reservoir refill

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 multiply-xor bijection with a Weyl key
// schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each 32 x 32 -> 64-bit product as one v_mad_u64_u32 (both halves at the cost of one quarter-rate
        // multiply; a low and a high multiply written apart are two)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u, p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // three-way XORs as single gfx950 three-input bit operations (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Correctly rounded square root for x >= 2^-96, +0 and +inf: the hardware estimate s (within 1 ulp) moved to
// a neighbour when the residual x - s' s of that neighbour s' (exact through fma) shows the square root is
// past the midpoint between them. This is the correction the compiler applies for sqrtf; its scaling of
// tiny inputs and its special-value fix-up are identities in this range, so the bits are sqrtf's.
__device__ __forceinline__ float sqrt_rn_big(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float sm = __uint_as_float(__float_as_uint(s) - 1u);
    const float sp = __uint_as_float(__float_as_uint(s) + 1u);
    const float rm = __builtin_fmaf(-sm, s, x);
    const float rp = __builtin_fmaf(-sp, s, x);
    float r = rm <= 0.0f ? sm : s;
    r = rp > 0.0f ? sp : r;
    return r;
}

// sqrtf(x) for x >= 0 (or +inf): sqrt_rn_big, unless a lane of the wave holds 0 < x < 2^-96, when the whole
// wave takes sqrtf (a wave-uniform branch, so the common case pays one compare)
__device__ __forceinline__ float sqrt_rn(float x) {
    if (__builtin_expect(__ballot(x > 0.0f && x < 0x1p-96f) != 0ull, 0)) return sqrtf(x);
    return sqrt_rn_big(x);
}

// a / b correctly rounded, for b in [2^-40, 2^40] and a = 0 or |a| in [2^-40, 2^40]: the compiler's division
// sequence (hardware reciprocal, one Newton step on it, two fma-corrected quotient steps) without its operand
// scaling and its special-value fix-up. Both are identities for such operands (no operand or quotient near the
// subnormal or overflow range, exponents less than 96 apart), so the bits are those of a / b.
__device__ __forceinline__ float div_rn_mid(float a, float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    const float r1 = __builtin_fmaf(__builtin_fmaf(-b, r, 1.0f), r, r);
    const float q0 = a * r1;
    const float q1 = __builtin_fmaf(__builtin_fmaf(-b, q0, a), r1, q0);
    return __builtin_fmaf(__builtin_fmaf(-b, q1, a), r1, q1);
}

// x in [2^-80, 2^80] (one unsigned compare of the bits; NaN and negative x fall outside), so that
// sqrt_rn_big(x) lies in [2^-40, 2^40]
__device__ __forceinline__ bool mid_range(float x) {
    return __float_as_uint(x) - 0x17800000u <= 0x67800000u - 0x17800000u;
}

// q / sqrtf(x), both correctly rounded, for x > 0 and q = 0 or |q| in [2^-40, 2^40]: sqrt_rn_big and div_rn_mid
// when every active lane of the wave has x in [2^-80, 2^80] (a wave-uniform branch), else sqrtf and the
// compiler's division
__device__ __forceinline__ float div_sqrt_rn(float q, float x) {
    if (__builtin_expect(__ballot(!mid_range(x)) != 0ull, 0)) return q / sqrtf(x);
    return div_rn_mid(q, sqrt_rn_big(x));
}

// 24 random bits m -> 2 (m 2^-24) - 1, uniform in [-1, 1). Both products are exact and so is the difference
// ((m - 2^23) 2^-23 needs at most 24 significant bits), so one fma gives the same bits.
__device__ __forceinline__ float signed_unit(uint32_t u) {
    return __builtin_fmaf((float)(u >> 8), 0x1p-23f, -1.0f);
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

// The same patch read from the DEM with a one-texel replicated border (row length Wp = W + 2 texels,
// row_bytes = 4 Wp) through a buffer resource: for (x, y) inside the grid the corner (floor(x - 1/2),
// floor(y - 1/2)) lies in [-1, W - 1] x [-1, H - 1], i.e. inside the padded grid, and the border holds
// exactly the clamped texels, so the four values and the arithmetic are those of bilinear().
__device__ __forceinline__ Sample bilinear_pad(__amdgpu_buffer_rsrc_t rs, uint32_t Wp, uint32_t row_bytes, float x,
                                               float y) {
    const float sx = x - 0.5f, sy = y - 0.5f;
    const float fc = floorf(sx), fr = floorf(sy);
    const float fx = sx - fc, fy = sy - fr;
    const uint32_t off = (__umul24((uint32_t)((int)fr + 1), Wp) + (uint32_t)((int)fc + 1)) * 4u;
    // two 8-byte loads (the raw words of a, b and of c, d), both issued before either is used
    const auto ab = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    const auto cd = __builtin_amdgcn_raw_buffer_load_b64(rs, off, row_bytes, 0);
    __builtin_amdgcn_sched_barrier(0);  // keep both loads ahead of their uses (one memory latency, not two)
    const float a = __uint_as_float(ab[0]), b = __uint_as_float(ab[1]);
    const float c = __uint_as_float(cd[0]), d = __uint_as_float(cd[1]);
    const float top = a + fx * (b - a);
    const float bot = c + fx * (d - c);
    Sample s;
    s.z = top + fy * (bot - top);
    s.gx = (b - a) + fy * ((d - c) - (b - a));
    s.gy = bot - top;
    return s;
}

// buffer resource over `bytes` bytes at p (gfx9 descriptor word 3: 32-bit data format)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Corners and fractions of the bilinear patch (or splat) at (x, y), indices clamped to the grid.
struct Corners {
    int ca, cb, ra, rb;
    float fx, fy;
};
__device__ __forceinline__ Corners corners(int H, int W, float x, float y) {
    const float sx = x - 0.5f, sy = y - 0.5f;
    const float fc = floorf(sx), fr = floorf(sy);
    Corners k;
    k.fx = sx - fc;
    k.fy = sy - fr;
    const int c0 = (int)fc, r0 = (int)fr;
    k.ca = min(max(c0, 0), W - 1);
    k.cb = min(max(c0 + 1, 0), W - 1);
    k.ra = min(max(r0, 0), H - 1);
    k.rb = min(max(r0 + 1, 0), H - 1);
    return k;
}

// Start state of release texel `texel` of a release texture with mult x mult texels per DEM cell (row-major,
// W * mult wide): its centre ((c + 1/2) / mult, (r + 1/2) / mult) in DEM cell units (mult = 1: the centre of
// DEM cell `texel`), the bilinear sample there and the unit direction of steepest descent (zero on flat
// ground). `cell` keeps the texel index, which keys the particle's random stream.
__device__ __forceinline__ StartRec start_state(const float* __restrict__ dem, int H, int W, uint32_t mult,
                                                uint32_t texel) {
    StartRec st;
    const uint32_t Wf = (uint32_t)W * mult;
    const uint32_t r = texel / Wf;
    const uint32_t c = texel - r * Wf;
    const float fm = (float)mult;
    st.x = ((float)c + 0.5f) / fm;
    st.y = ((float)r + 0.5f) / fm;
    const Sample s0 = bilinear(dem, H, W, st.x, st.y);
    st.z = s0.z;
    st.gx = s0.gx;
    st.gy = s0.gy;
    const float gg = s0.gx * s0.gx + s0.gy * s0.gy;
    if (gg > 0.0f) {
        const float t = 1.0f / sqrtf(gg);
        st.dx = -(s0.gx * t);
        st.dy = -(s0.gy * t);
    } else {
        st.dx = 0.0f;
        st.dy = 0.0f;
    }
    st.cell = texel;
    return st;
}

// start state at the centre of DEM cell `cell`, with the patch read from the padded DEM (the same values, so the same result)
__device__ __forceinline__ StartRec start_state_pad(__amdgpu_buffer_rsrc_t rs, uint32_t Wp, uint32_t row_bytes, int W,
                                                    uint32_t cell) {
    StartRec st;
    const int r = (int)(cell / (uint32_t)W);
    const int c = (int)(cell - (uint32_t)r * (uint32_t)W);
    st.x = (float)c + 0.5f;
    st.y = (float)r + 0.5f;
    const Sample s0 = bilinear_pad(rs, Wp, row_bytes, st.x, st.y);
    st.z = s0.z;
    st.gx = s0.gx;
    st.gy = s0.gy;
    const float gg = s0.gx * s0.gx + s0.gy * s0.gy;
    if (gg > 0.0f) {
        const float t = 1.0f / sqrtf(gg);
        st.dx = -(s0.gx * t);
        st.dy = -(s0.gy * t);
    } else {
        st.dx = 0.0f;
        st.dy = 0.0f;
    }
    st.cell = cell;
    return st;
}

__device__ __forceinline__ uint32_t udiv(uint32_t n, const DivU32& d) {
    const uint32_t t = __umulhi(d.mul, n);
    return (t + ((n - t) >> d.sh1)) >> d.sh2;
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

__device__ __forceinline__ float uniform_f(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ uint32_t uniform_u(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The run constants held in scalar registers (every lane has the same run).
__device__ __forceinline__ RunConst uniform_run(const RunConst& r) {
    RunConst u = r;
    u.per = uniform_f(r.per);
    u.Q = uniform_f(r.Q);
    u.rnd = uniform_f(r.rnd);
    u.L = uniform_f(r.L);
    u.dl2 = uniform_f(r.dl2);
    u.mdl = uniform_f(r.mdl);
    u.cd = uniform_f(r.cd);
    u.tca = uniform_f(r.tca);
    u.key0 = uniform_u(r.key0);
    u.key1 = uniform_u(r.key1);
    u.run = uniform_u(r.run);
    u.use_alpha = uniform_u(r.use_alpha);
    u.dem_off = uniform_u(r.dem_off);
    u.cells_off = uniform_u(r.cells_off);
    u.raster_off = uniform_u(r.raster_off);
    u.P = uniform_u(r.P);
    u.n_slots = ((unsigned long long)uniform_u((uint32_t)(r.n_slots >> 32)) << 32) | uniform_u((uint32_t)r.n_slots);
    // the DEM tile's offset builds the buffer resource of every gather: a value the compiler cannot prove
    // uniform there makes each buffer load a loop over the distinct resources of the wave's lanes
    u.pad_off = uniform_u(r.pad_off);
    u.use_rec = uniform_u(r.use_rec);
    return u;
}

// Run holding padded slot `slot`: the r with run_off[r] <= slot < run_off[r + 1]. Wave-uniform input.
__device__ __forceinline__ uint32_t find_run(const unsigned long long* __restrict__ off, uint32_t n_runs,
                                             uint64_t slot) {
    uint32_t lo = 0, hi = n_runs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= slot)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// start of XCD partition p of the padded slot range [0, total): a multiple of kChunk
__device__ __forceinline__ uint64_t part_begin(uint64_t total, uint32_t p) {
    if (p >= (uint32_t)kXcds) return total;
    return (total / kChunk * p / kXcds) * kChunk;
}

// Blocks of a persistent grid that take part for `total` slots: enough for about `spl` (default
// kSlotsPerLane) slots per lane, at least one per XCD (measured: a 640,000-particle pass runs 2.3x faster on 8 slots per lane
// than on the full grid's ~1).
constexpr uint64_t kSlotsPerLane = 8;
__device__ __forceinline__ uint64_t active_blocks(uint64_t total, int block_threads, uint32_t spl = kSlotsPerLane) {
    const uint64_t per_block = (uint64_t)block_threads * (spl ? spl : 1u);
    const uint64_t want = (total + per_block - 1) / per_block;
    return want > (uint64_t)kXcds ? want : (uint64_t)kXcds;
}

// Wave-uniform slot dispenser of the smooth kernels. The first chunks of 64 slots are dealt out without
// atomics, round-robin over the grid's waves (kStaticShare of the chunks, a whole number of rounds); the
// rest come from per-XCD queues, the wave starting on its own XCD's partition of the remainder and moving
// on when it is empty. Device-scope atomics on one counter are serialised at the memory side: taking
// every chunk from the queues cost each wave 4.5-10 us per take (up to ~150 waves per counter). The
// counters sit kQueueStride words apart, each in a memory line of its own.
constexpr uint32_t kStaticShareNum = 3, kStaticShareDen = 4;
struct Dispenser {
    uint64_t total;      // padded slot count (a multiple of kChunk)
    uint64_t dyn_begin;  // slots below it are dealt out statically
    uint64_t st_next;    // the wave's next static chunk (>= dyn_begin: none left)
    uint64_t st_stride;  // kChunk x the grid's waves
    uint32_t part, tried;
    bool queue_empty;
    uint64_t res_next, res_end;

    // `wave`: the wave's index among the `waves` waves of the grid that take part
    __device__ __forceinline__ void init(uint64_t total_slots, uint32_t xcd, uint64_t wave, uint64_t waves) {
        total = total_slots;
        const uint64_t chunks = total / kChunk;
        const uint64_t rounds = waves ? chunks * kStaticShareNum / kStaticShareDen / waves : 0;
        dyn_begin = rounds * waves * kChunk;
        st_stride = waves * kChunk;
        st_next = rounds ? wave * kChunk : dyn_begin;
        part = xcd;
        tried = 0;
        queue_empty = dyn_begin >= total;
        res_next = res_end = 0;
    }
    __device__ __forceinline__ bool drained() const {
        return queue_empty && st_next >= dyn_begin && res_next >= res_end;
    }

    // Hands slots to the idle lanes (ballot `idle`) in lane order; returns this lane's slot or ~0.
    __device__ __forceinline__ uint64_t take(unsigned long long* __restrict__ queues, uint64_t idle, int lane,
                                             uint64_t below) {
        const int nidle = __popcll(idle);
        const uint64_t avail = res_end - res_next;
        const int rank = __popcll(idle & below);
        uint64_t slot = ~0ull;
        if (avail >= (uint64_t)nidle) {
            slot = res_next + rank;
            res_next += nidle;
            return slot;
        }
        uint64_t base = 0, cend = 0;
        if (st_next < dyn_begin) {
            base = st_next;
            cend = base + kChunk;
            st_next += st_stride;
        } else {
            const int leader = __ffsll((long long)idle) - 1;
            const uint64_t rem = total - dyn_begin;
            while (!queue_empty) {
                const uint64_t pb = dyn_begin + part_begin(rem, part), pe = dyn_begin + part_begin(rem, part + 1);
                uint64_t got = 0;
                if (lane == leader) got = atomicAdd(queues + part * kQueueStride, (unsigned long long)kChunk);
                got = wave_bcast64(__shfl(got, leader, kWave));
                if (pb + got < pe) {
                    base = pb + got;
                    cend = (base + kChunk < pe) ? base + kChunk : pe;
                    break;
                }
                part = (part + 1) % kXcds;
                if (++tried >= (uint32_t)kXcds) queue_empty = true;
            }
        }
        if ((uint64_t)rank < avail)
            slot = res_next + rank;
        else if (base + (rank - avail) < cend)
            slot = base + (rank - avail);
        const uint64_t next = base + ((uint64_t)nidle - avail);
        res_next = next < cend ? next : cend;
        res_end = cend;
        return slot;
    }
};

}  // namespace dev
}  // namespace avl
