// Smooth variant of the trajectory pass and its adjoint (arXiv 2506.23364, section 5.2: the particles
// spread the released mass along the flow; here the mass each particle carries is deposited where it
// comes to rest, so the deposit raster is a differentiable function of the friction parameters).
//
// Forward: every particle of release cell c carries mp = mass[c] / P. An energy stop during a step puts
// it at the zero of the step's (linear) energy numerator, the fraction t* = v^2 / (v^2 - num) of the
// step; a runout-angle stop or the step limit leaves it where it is; leaving the grid loses the mass.
// The mass is splatted bilinearly (the height patch's corners and weights) into an int64 fixed-point
// raster (2^-24 units): order-independent, so reproducible bit for bit. Optionally every accepted step
// splats mp * v at the new position (velocity raster). Every kCkpt steps the particle's state
// (x, y, dx, dy, v^2) is checkpointed, and its end (steps done, reason) is recorded.
//
// Adjoint, per particle: the paths do not depend on (mu, xi, h, mass), so only v^2 along the path and
// the fractional last step do. Given gD = dL/dD, the kernel recomputes the last segment from its
// checkpoint, takes dL/dp* through the splat weights and dL/dt* = dL/dp* . (p1 - p), then runs the
// reverse sweep of the v^2 recursion segment by segment (each segment recomputed forward from its
// checkpoint into a per-lane scratch of (a_k, v^2_{k+1}), then swept backward). Per-particle
// results are reduced in a fixed order (deterministic).
#include "particle.h"

namespace avl {

using namespace dev;

namespace {

constexpr uint32_t kCkpt = 64;        // steps between checkpoints (even: segments start on even steps)
constexpr int kSmoothBlock = 256;
constexpr int kBackwardGrid = 1536;   // blocks of the adjoint kernel (its scratch is sized for this): six waves
                                      // per SIMD; 1024 (four) left the long paths' recompute short of waves
constexpr int kReduceChunk = 4096;    // particles per block of the gradient reduction
static_assert(kCkpt % 2 == 0, "segments must start on even steps (one Philox block serves two steps)");

enum : uint32_t { kEndLimit = 0, kEndExit = 1, kEndStop = 2, kEndAngle = 3 };
enum : int { kAccept = 0, kExit = 1, kStop = 2, kAngle = 3 };

struct State {
    float x, y, z, gx, gy, dx, dy, v2, x0, y0, zr;
    uint32_t spare_x, spare_y;
};

struct StepOut {
    int outcome;
    float x1, y1, num;  // target of the step and its energy numerator
    float a;            // drag term a = 2g ds / (xi h) of an accepted step
};

// The DEM with its replicated border, read through a buffer resource (no clamps, 32-bit offsets, both
// rows of the patch in flight), as in the plain pass; the same values as the clamped patch.
struct PadDem {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t Wp, row_bytes;
};

__device__ __forceinline__ PadDem pad_dem(const SmoothArgs& a) {
    PadDem d;
    d.rs = buffer_rsrc(a.dem_pad, a.pad_bytes);
    d.Wp = (uint32_t)a.W + 2u;
    d.row_bytes = 4u * d.Wp;
    return d;
}

__device__ __forceinline__ Sample sample(const PadDem& d, float x, float y) {
    return bilinear_pad(d.rs, d.Wp, d.row_bytes, x, y);
}

// Step n of the model (the same binary32 operations as the plain pass). Updates s when accepted. `even`
// is n's parity (a wave-uniform value where every live particle of the wave has the parity of the wave's
// iteration, which makes the Philox block a uniform branch).
__device__ __forceinline__ StepOut step(State& s, uint32_t n, uint32_t rep, uint32_t cell_id, const RunConst& rc,
                                        const PadDem& dem, int H, int W, float g2, bool even) {
    StepOut o;
    uint32_t ux, uy;
    if (even) {
        const uint4 b = philox4x32_10(n >> 1, rep, cell_id, rc.run, rc.key0, rc.key1);
        ux = b.x;
        uy = b.y;
        s.spare_x = b.z;
        s.spare_y = b.w;
    } else {
        ux = s.spare_x;
        uy = s.spare_y;
    }
    const float rx = signed_unit(ux), ry = signed_unit(uy);
    const float gg = s.gx * s.gx + s.gy * s.gy;
    const float t = gg > 0.0f ? div_sqrt_rn(rc.Q, gg) : 0.0f;  // Q = 1 - persistence: 0 or in [2^-24, 1]
    const float wx = (rc.per * s.dx - t * s.gx) + rc.rnd * rx;
    const float wy = (rc.per * s.dy - t * s.gy) + rc.rnd * ry;
    const float ww = wx * wx + wy * wy;
    if (ww > 0.0f) {
        const float inv = div_sqrt_rn(1.0f, ww);
        s.dx = wx * inv;
        s.dy = wy * inv;
    }
    o.x1 = s.x + rc.L * s.dx;
    o.y1 = s.y + rc.L * s.dy;
    // Every lane runs the whole step and the outcome selects what it keeps (no branch per outcome, so the
    // compiler copies no state at their joins): a target off the grid is read through the buffer's bounds
    // check, which cannot fault; its values are discarded.
    const float fc1 = floorf(o.x1), fr1 = floorf(o.y1);
    const bool inb = fc1 >= 0.0f && fc1 < (float)W && fr1 >= 0.0f && fr1 < (float)H;
    const Sample s1 = sample(dem, o.x1, o.y1);
    const float dz = s.z - s1.z;
    // dl2 + dz^2 >= dl2: with dl2 >= 2^-96 (a run constant) no lane needs the small-argument check
    float ds;
    if (rc.dl2 >= 0x1p-96f)
        ds = sqrt_rn_big(rc.dl2 + dz * dz);
    else
        ds = sqrt_rn(rc.dl2 + dz * dz);
    const float num = s.v2 + g2 * (dz - rc.mdl);
    const bool pos = num > 0.0f;
    const float aa = rc.cd * ds;
    const float v2n = num / (1.0f + aa);
    bool angle = false;
    if (rc.use_alpha) {
        const float hx = o.x1 - s.x0, hy = o.y1 - s.y0;
        angle = (s.zr - s1.z) < rc.tca * sqrtf(hx * hx + hy * hy);
    }
    o.num = inb ? num : 0.0f;
    o.a = (inb && pos) ? aa : 0.0f;
    o.outcome = !inb ? kExit : (!pos ? kStop : (angle ? kAngle : kAccept));
    const bool acc = inb && pos && !angle;
    s.x = acc ? o.x1 : s.x;
    s.y = acc ? o.y1 : s.y;
    s.z = acc ? s1.z : s.z;
    s.gx = acc ? s1.gx : s.gx;
    s.gy = acc ? s1.gy : s.gy;
    s.v2 = acc ? v2n : s.v2;
    return o;
}

__device__ __forceinline__ void splat_q(unsigned long long* __restrict__ q, int H, int W, float x, float y, float val) {
    const Corners k = corners(H, W, x, y);
    const float w00 = (1.0f - k.fx) * (1.0f - k.fy), w01 = k.fx * (1.0f - k.fy);
    const float w10 = (1.0f - k.fx) * k.fy, w11 = k.fx * k.fy;
    const float sc = 16777216.0f;  // 2^24
    atomicAdd(q + (size_t)k.ra * W + k.ca, (unsigned long long)(long long)rintf((val * w00) * sc));
    atomicAdd(q + (size_t)k.ra * W + k.cb, (unsigned long long)(long long)rintf((val * w01) * sc));
    atomicAdd(q + (size_t)k.rb * W + k.ca, (unsigned long long)(long long)rintf((val * w10) * sc));
    atomicAdd(q + (size_t)k.rb * W + k.cb, (unsigned long long)(long long)rintf((val * w11) * sc));
}

// Workgroup table of the forward's deposit: the particles of a block come from neighbouring release cells
// and come to rest in overlapping cells, so their splats are summed in LDS (int64, order-independent like
// the raster) and each touched cell reaches the raster with one atomic when the block ends. A corner
// whose probe window is taken goes to the raster directly.
constexpr int kDepLog2 = 12;
constexpr int kDepSlots = 1 << kDepLog2;  // 4096 x (4-byte tag + 8-byte sum) = 48 KB
constexpr int kDepProbes = 4;
constexpr uint32_t kDepEmpty = 0xFFFFFFFFu;

struct DepTable {
    uint32_t tag[kDepSlots];
    unsigned long long val[kDepSlots];
};

__device__ __forceinline__ uint32_t dep_home(uint32_t cell) { return (cell * 2654435761u) >> (32 - kDepLog2); }

// The table's adds name the LDS address space: the compiler would otherwise merge them with the raster's
// fallback add into one generic (flat) atomic through a selected pointer, which every later LDS wait and
// every vector-memory wait then has to wait for.
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ __forceinline__ void lds_add_u64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add((lds_u64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t dep_tag(DepTable& t, uint32_t k) {
    return __hip_atomic_load(&t.tag[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds v to the table slot of `cell` (claimed if a probe finds an empty slot first), else to the raster.
// `first` is a read of the cell's home slot: slots only ever go from empty to a tag, so a stale read of it
// is either right or empty, and an empty read is settled by the claim.
__device__ __forceinline__ void dep_add(DepTable& t, unsigned long long* __restrict__ q, uint32_t cell,
                                        unsigned long long v, uint32_t first) {
    if (v == 0ull) return;
    const uint32_t h = dep_home(cell);
    for (int p = 0; p < kDepProbes; ++p) {
        const uint32_t k = (h + (uint32_t)p) & (uint32_t)(kDepSlots - 1);
        uint32_t cur = p == 0 ? first : dep_tag(t, k);
        if (cur == kDepEmpty) cur = atomicCAS(&t.tag[k], kDepEmpty, cell);  // the old tag: empty if taken here
        if (cur == kDepEmpty || cur == cell) {
            lds_add_u64(&t.val[k], v);
            return;
        }
    }
    atomicAdd(q + cell, v);
}

// splat_q through the block's table; the home slots of the four corners are read together (one LDS round
// trip instead of four)
__device__ __forceinline__ void splat_q_table(DepTable& t, unsigned long long* __restrict__ q, int H, int W, float x,
                                              float y, float val) {
    const Corners k = corners(H, W, x, y);
    const float w00 = (1.0f - k.fx) * (1.0f - k.fy), w01 = k.fx * (1.0f - k.fy);
    const float w10 = (1.0f - k.fx) * k.fy, w11 = k.fx * k.fy;
    const float sc = 16777216.0f;  // 2^24
    const uint32_t c00 = (uint32_t)(k.ra * W + k.ca), c01 = (uint32_t)(k.ra * W + k.cb);
    const uint32_t c10 = (uint32_t)(k.rb * W + k.ca), c11 = (uint32_t)(k.rb * W + k.cb);
    const uint32_t f00 = dep_tag(t, dep_home(c00)), f01 = dep_tag(t, dep_home(c01));
    const uint32_t f10 = dep_tag(t, dep_home(c10)), f11 = dep_tag(t, dep_home(c11));
    dep_add(t, q, c00, (unsigned long long)(long long)rintf((val * w00) * sc), f00);
    dep_add(t, q, c01, (unsigned long long)(long long)rintf((val * w01) * sc), f01);
    dep_add(t, q, c10, (unsigned long long)(long long)rintf((val * w10) * sc), f10);
    dep_add(t, q, c11, (unsigned long long)(long long)rintf((val * w11) * sc), f11);
}

__device__ __forceinline__ float mass_per_particle(const float* __restrict__ mass, uint32_t cell, uint32_t P) {
    return (mass ? mass[cell] : 1.0f) / (float)P;
}

// release cell of particle slot `slot`, and the particle's replica index within it
__device__ __forceinline__ uint64_t cell_of_slot(uint64_t slot, const SmoothArgs& a, uint32_t P, uint32_t* rep) {
    const uint64_t i = (slot >> 32) == 0 ? (uint64_t)udiv((uint32_t)slot, a.pdiv) : slot / P;
    *rep = (uint32_t)(slot - i * P);
    return i;
}

}  // namespace

__global__ __launch_bounds__(256) void k_particle_mass(const float* __restrict__ mass, const int32_t* __restrict__ cells,
                                                       const int32_t* __restrict__ n_cells, int64_t cap,
                                                       uint32_t P, float* __restrict__ mpc) {
    const int64_t n = min((int64_t)*n_cells, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mpc[i] = mass_per_particle(mass, (uint32_t)cells[i], P);
}

hipError_t launch_particle_mass(const float* mass, const int32_t* cells, const int32_t* n_cells, int64_t cap,
                                uint32_t P, float* mpc, hipStream_t s) {
    const int64_t blocks = (cap + 255) / 256;
    hipLaunchKernelGGL(k_particle_mass, dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)), dim3(256),
                       0, s, mass, cells, n_cells, cap, P > 0 ? P : 1u, mpc);
    return hipGetLastError();
}


// kBlk threads per block share one deposit table; a.spl particle slots per lane size the grid of a small
// problem (its variants: 256 threads at 8 slots per lane suit short paths, larger blocks at 2 long ones).
template <int kBlk>
__global__ __launch_bounds__(kBlk) void k_smooth_forward(SmoothArgs a) {
    if ((uint64_t)blockIdx.x >= active_blocks(a.run_off[1], kBlk, a.spl)) return;  // small problems: fewer blocks
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const RunConst rc = uniform_run(a.runs[0]);
    const int H = a.H, W = a.W;
    const PadDem dd = pad_dem(a);
    Dispenser disp;
    {
        const uint64_t total = wave_bcast64(a.run_off[1]);
        const uint64_t nb = min((uint64_t)gridDim.x, active_blocks(total, blockDim.x, a.spl));
        const uint32_t wpb = blockDim.x / kWave;
        disp.init(total, xcd_id(), (uint64_t)blockIdx.x * wpb + threadIdx.x / kWave, nb * wpb);
    }
    const size_t cplane = (size_t)a.C * a.cap;
    __shared__ DepTable dep;
    for (int k = threadIdx.x; k < kDepSlots; k += kBlk) {
        dep.tag[k] = kDepEmpty;
        dep.val[k] = 0ull;
    }
    __syncthreads();

    bool alive = false;
    State s{};
    uint32_t n = 0, rep = 0, cell_id = 0;
    uint64_t slot_id = 0;
    float mp = 0.0f;
    uint64_t st_steps = 0;
    uint32_t st_exit = 0, st_stop = 0, st_limit = 0;
    // Particles start on the wave's even iterations only: a live particle's step count then has the parity
    // of the wave's iteration, so the Philox block (one per two steps) is a uniform branch, and the slot
    // hand-out runs every other iteration. A particle starts from its release cell's start record (one
    // load, the mass per particle beside it). The waits for vector memory cover stores as well as loads,
    // so an end record is written in the iteration after the particle ended, after the hand-out's loads.
    bool end_pending = false;
    uint64_t end_slot = 0;
    uint32_t end_val = 0;
    auto end_particle = [&](uint32_t why) {
        end_pending = true;
        end_slot = slot_id;
        end_val = (n << 2) | why;
        alive = false;
    };

    for (uint32_t wit = 0;; ++wit) {
        const bool even = (wit & 1u) == 0u;
        if (even) {
            const uint64_t idle = __ballot(!alive);
            if (__popcll(idle) == kWave && disp.drained() && __ballot(end_pending) == 0ull) break;
            if (idle && !disp.drained()) {
                const uint64_t slot = disp.take(a.queues, idle, lane, below);
                if (!alive && slot < rc.n_slots) {
                    const uint64_t i = cell_of_slot(slot, a, rc.P, &rep);
                    const StartRec st = a.starts[i];
                    mp = a.mpc[i];
                    s.x = st.x;
                    s.y = st.y;
                    s.z = st.z;
                    s.gx = st.gx;
                    s.gy = st.gy;
                    s.dx = st.dx;
                    s.dy = st.dy;
                    s.x0 = st.x;
                    s.y0 = st.y;
                    s.zr = st.z;
                    s.v2 = 0.0f;
                    cell_id = st.cell;
                    slot_id = slot;
                    n = 0;
                    alive = true;
                }
            }
        }
        if (end_pending) {
            a.end_rec[end_slot] = end_val;
            end_pending = false;
        }
        if (!alive) continue;
        if (n >= a.S) {
            ++st_limit;
            splat_q_table(dep, a.dep_q, H, W, s.x, s.y, mp);
            end_particle(kEndLimit);
            continue;
        }
        if (n != 0 && n % kCkpt == 0) {  // checkpoint 0 is the release cell's start record
            const size_t at = (size_t)(n / kCkpt) * a.cap + slot_id;
            a.ck[at] = s.x;
            a.ck[cplane + at] = s.y;
            a.ck[2 * cplane + at] = s.dx;
            a.ck[3 * cplane + at] = s.dy;
            a.ck[4 * cplane + at] = s.v2;
        }
        ++st_steps;
        const float xp = s.x, yp = s.y, v2p = s.v2;
        const StepOut o = step(s, n, rep, cell_id, rc, dd, H, W, a.g2, even);
        if (o.outcome == kAccept) {
            ++n;
            if (a.vel_q) splat_q(a.vel_q, H, W, s.x, s.y, mp * sqrtf(s.v2));
            continue;
        }
        if (o.outcome == kExit) {
            ++st_exit;
            end_particle(kEndExit);
        } else if (o.outcome == kStop) {
            ++st_stop;
            const float t = v2p > 0.0f ? v2p / (v2p - o.num) : 0.0f;
            splat_q_table(dep, a.dep_q, H, W, xp + t * (o.x1 - xp), yp + t * (o.y1 - yp), mp);
            end_particle(kEndStop);
        } else {
            ++st_stop;
            splat_q_table(dep, a.dep_q, H, W, xp, yp, mp);
            end_particle(kEndAngle);
        }
    }
    // every wave of the block is done: the table's sums go to the raster, and the statistics, summed over
    // the block in LDS, go to the four counters with one atomic each per block (the counters share a
    // memory line, where device-scope atomics serialise)
    __shared__ unsigned long long bst[4];
    if (threadIdx.x < 4) bst[threadIdx.x] = 0ull;
    __syncthreads();
    const uint64_t s0 = wave_sum64(st_steps), s1 = wave_sum64(st_exit), s2 = wave_sum64(st_stop);
    const uint64_t s3 = wave_sum64(st_limit);
    if (lane == 0) {
        lds_add_u64(&bst[0], s0);
        lds_add_u64(&bst[1], s1);
        lds_add_u64(&bst[2], s2);
        lds_add_u64(&bst[3], s3);
    }
    for (int k = threadIdx.x; k < kDepSlots; k += kBlk)
        if (dep.tag[k] != kDepEmpty && dep.val[k] != 0ull) atomicAdd(a.dep_q + dep.tag[k], dep.val[k]);
    __syncthreads();
    if (threadIdx.x < 4 && bst[threadIdx.x]) atomicAdd(a.stats + threadIdx.x, bst[threadIdx.x]);
}

__global__ __launch_bounds__(kSmoothBlock) void k_smooth_backward(SmoothArgs a) {
    if ((uint64_t)blockIdx.x >= active_blocks(a.run_off[1], kSmoothBlock, a.spl)) return;  // small problems: fewer blocks
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const RunConst rc = uniform_run(a.runs[0]);
    const int H = a.H, W = a.W;
    const PadDem dd = pad_dem(a);
    const size_t T = (size_t)gridDim.x * blockDim.x;
    const size_t gtid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t cplane = (size_t)a.C * a.cap;
    const float g2dl = a.g2dl;
    const float xi = a.pdev ? a.pdev->xi : a.xi;  // a device-side loop keeps the parameters on the device
    Dispenser disp;
    {
        const uint64_t total = wave_bcast64(a.run_off[1]);
        const uint64_t nb = min((uint64_t)gridDim.x, active_blocks(total, blockDim.x, a.spl));
        const uint32_t wpb = blockDim.x / kWave;
        disp.init(total, xcd_id(), (uint64_t)blockIdx.x * wpb + threadIdx.x / kWave, nb * wpb);
    }

    for (;;) {
        const uint64_t idle = __ballot(true);
        if (disp.drained()) break;
        const uint64_t slot = disp.take(a.queues, idle, lane, below);
        if (slot >= rc.n_slots) continue;
        uint32_t rep = 0;
        const uint64_t i = cell_of_slot(slot, a, rc.P, &rep);
        const StartRec st = a.starts[i];  // the release state, as the forward started the particle
        const uint32_t cell_id = st.cell;
        const float mp = a.mpc[i];
        const uint32_t rec = a.end_rec[slot];
        const uint32_t n_end = rec >> 2, reason = rec & 3u;
        float dmu = 0.0f, dxi = 0.0f, dh = 0.0f, gw = 0.0f;
        if (reason != kEndExit) {
            // last segment: from its checkpoint (or the release) up to the end
            State s{};
            int32_t c_last = -1;
            if (a.C > 0) c_last = (int32_t)min(n_end / kCkpt, a.C - 1);
            uint32_t n0 = 0;
            auto load = [&](int32_t c) {
                s.x0 = st.x;
                s.y0 = st.y;
                s.zr = st.z;
                if (c <= 0) {  // the release (checkpoint 0 is the start record, v^2 = 0)
                    s.x = st.x;
                    s.y = st.y;
                    s.z = st.z;
                    s.gx = st.gx;
                    s.gy = st.gy;
                    s.dx = st.dx;
                    s.dy = st.dy;
                    s.v2 = 0.0f;
                    return;
                }
                const size_t at = (size_t)c * a.cap + slot;
                s.x = a.ck[at];
                s.y = a.ck[cplane + at];
                s.dx = a.ck[2 * cplane + at];
                s.dy = a.ck[3 * cplane + at];
                s.v2 = a.ck[4 * cplane + at];
                const Sample sm = sample(dd, s.x, s.y);
                s.z = sm.z;
                s.gx = sm.gx;
                s.gy = sm.gy;
            };
            load(c_last);
            n0 = c_last < 0 ? 0u : (uint32_t)c_last * kCkpt;
            // segments start at checkpoints, multiples of kCkpt (even): the step's parity is that of the trip
            // count, the same for every lane still in the loop
            for (uint32_t t = 0; n0 + t < n_end; ++t) {
                const StepOut o = step(s, n0 + t, rep, cell_id, rc, dd, H, W, a.g2, (t & 1u) == 0u);
                a.scratch[(size_t)t * T + gtid] = make_float2(o.a, s.v2);
            }
            float px = s.x, py = s.y;
            float lam = 0.0f, gt = 0.0f;
            bool stop = false;
            if (reason == kEndStop) {
                const float xp = s.x, yp = s.y, v2p = s.v2;
                const StepOut o = step(s, n_end, rep, cell_id, rc, dd, H, W, a.g2, (n_end & 1u) == 0u);
                const float t = v2p > 0.0f ? v2p / (v2p - o.num) : 0.0f;
                px = xp + t * (o.x1 - xp);
                py = yp + t * (o.y1 - yp);
                // dL/dp* through the splat weights, dL/dt*
                const Corners k = corners(H, W, px, py);
                const float g00 = a.gD[(size_t)k.ra * W + k.ca], g01 = a.gD[(size_t)k.ra * W + k.cb];
                const float g10 = a.gD[(size_t)k.rb * W + k.ca], g11 = a.gD[(size_t)k.rb * W + k.cb];
                const float gpx = ((g01 - g00) * (1.0f - k.fy)) + ((g11 - g10) * k.fy);
                const float gpy = ((g10 - g00) * (1.0f - k.fx)) + ((g11 - g01) * k.fx);
                const float w00 = (1.0f - k.fx) * (1.0f - k.fy), w01 = k.fx * (1.0f - k.fy);
                const float w10 = (1.0f - k.fx) * k.fy, w11 = k.fx * k.fy;
                gw = ((g00 * w00) + (g01 * w01)) + ((g10 * w10) + (g11 * w11));
                gt = mp * ((gpx * (o.x1 - xp)) + (gpy * (o.y1 - yp)));
                const float Dn = v2p - o.num;
                if (Dn > 0.0f) {
                    lam = gt / Dn;
                    dmu = -((gt * (v2p / Dn)) * (g2dl / Dn));
                }
                stop = true;
            } else {
                const Corners k = corners(H, W, px, py);
                const float g00 = a.gD[(size_t)k.ra * W + k.ca], g01 = a.gD[(size_t)k.ra * W + k.cb];
                const float g10 = a.gD[(size_t)k.rb * W + k.ca], g11 = a.gD[(size_t)k.rb * W + k.cb];
                const float w00 = (1.0f - k.fx) * (1.0f - k.fy), w01 = k.fx * (1.0f - k.fy);
                const float w10 = (1.0f - k.fx) * k.fy, w11 = k.fx * k.fy;
                gw = ((g00 * w00) + (g01 * w01)) + ((g10 * w10) + (g11 * w11));
            }
            if (stop) {
                // reverse sweep: the last segment from the scratch, then earlier segments recomputed
                // an energy stop needs a step, so step_limit >= 1 and checkpoint 0 exists: c_last >= 0
                for (int32_t c = c_last; c >= 0; --c) {
                    const uint32_t c0 = (uint32_t)c * kCkpt;
                    const uint32_t c1 = (c == c_last) ? n_end : c0 + kCkpt;
                    if (c != c_last) {
                        load(c);
                        for (uint32_t t = 0; c0 + t < c1; ++t) {
                            const StepOut o = step(s, c0 + t, rep, cell_id, rc, dd, H, W, a.g2, (t & 1u) == 0u);
                            a.scratch[(size_t)t * T + gtid] = make_float2(o.a, s.v2);
                        }
                    }
                    for (uint32_t k = c1; k-- > c0;) {
                        const float2 e = a.scratch[(size_t)(k - c0) * T + gtid];
                        const float aa = e.x, v2n = e.y;
                        const float op = 1.0f + aa;
                        dmu = dmu - lam * (g2dl / op);
                        dxi = dxi + lam * ((v2n * aa) / (xi * op));
                        dh = dh + lam * ((v2n * aa) / (a.h * op));
                        lam = lam / op;
                    }
                }
            }
        }
        a.pp[slot] = dmu;
        a.pp[a.cap + slot] = dxi;
        a.pp[2 * a.cap + slot] = dh;
        a.pp[3 * a.cap + slot] = gw;
    }
}

// ------------------------------------------------------------------------------------------ reductions

// Sum of the per-particle (dmu, dxi, dh) over particles [0, n): each block sums kReduceChunk particles
// (16 per thread in order, then a fixed tree) into partial[block]; all in binary64.
__global__ __launch_bounds__(256) void k_reduce_params(const float* __restrict__ pp, unsigned long long cap,
                                                       const RunConst* __restrict__ runs, double* __restrict__ part) {
    __shared__ double sh[3][256];
    const unsigned long long n = runs[0].n_slots;
    const unsigned long long base = (unsigned long long)blockIdx.x * kReduceChunk + threadIdx.x * 16ull;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 16; ++k) {
        const unsigned long long i = base + k;
        if (i < n) {
            acc[0] += (double)pp[i];
            acc[1] += (double)pp[cap + i];
            acc[2] += (double)pp[2 * cap + i];
        }
    }
    for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[3 * (size_t)blockIdx.x + q] = sh[q][0];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int q = 0; q < 3; ++q) acc[q] += part[3 * (size_t)b + q];
    for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[q] = sh[q][0];
}

// dL/dmass of release cell i: (sum over its P particles of sum gD w, in order, binary64) / P
__global__ __launch_bounds__(256) void k_dmass(const float* __restrict__ gw, const int32_t* __restrict__ cells,
                                               const int32_t* __restrict__ n_cells, const RunConst* __restrict__ runs,
                                               float* __restrict__ dmass) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (runs[0].n_slots == 0 || i >= (int64_t)*n_cells) return;
    const uint32_t P = runs[0].P;
    double s = 0.0;
    for (uint32_t j = 0; j < P; ++j) s += (double)gw[(size_t)i * P + j];
    dmass[cells[i]] = (float)(s / (double)P);
}

// fixed point (2^-24) -> float
__global__ __launch_bounds__(256) void k_q_to_float(const unsigned long long* __restrict__ q, int64_t n,
                                                    float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)((double)(long long)q[i] * 0x1p-24);
}

// ------------------------------------------------------------------------------------------ calibration loss
// L = sum (D - T)^2 / N and dL/dD = c (D - T), c = 2/N rounded to binary32. The differences are binary32;
// their squares are exact in binary64 and summed in a fixed order (per thread over a fixed grid stride,
// then over the wave, the block, and the kMseBlocks block sums), so L does not depend on timing.
constexpr int kMseBlocks = 1024;
constexpr int kMseThreads = 256;

__device__ __forceinline__ double block_sum_f64(double v, double* lds) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) t += lds[k];
    return t;  // valid in thread 0
}

__global__ __launch_bounds__(kMseThreads) void k_mse_partial(const float* __restrict__ dep,
                                                           const float* __restrict__ tgt, int64_t n, float c,
                                                           float* __restrict__ gD, double* __restrict__ part) {
    __shared__ double lds[kMseThreads / kWave];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kMseThreads + threadIdx.x; i < n; i += (int64_t)kMseBlocks * kMseThreads) {
        const float d = dep[i] - tgt[i];
        gD[i] = c * d;
        acc += (double)d * (double)d;
    }
    const double t = block_sum_f64(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kMseThreads) void k_mse_final(const double* __restrict__ part, double n,
                                                         double* __restrict__ loss) {
    __shared__ double lds[kMseThreads / kWave];
    double acc = 0.0;
    for (int k = threadIdx.x; k < kMseBlocks; k += kMseThreads) acc += part[k];
    const double t = block_sum_f64(acc, lds);
    if (threadIdx.x == 0) *loss = t / n;
}

hipError_t launch_mse_grad(const float* dep, const float* target, int64_t n, float c, float* gD, double* part,
                           double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mse_partial, dim3(kMseBlocks), dim3(kMseThreads), 0, s, dep, target, n, c, gD, part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(kMseThreads), 0, s, part, (double)n, loss);
    return hipGetLastError();
}

size_t mse_partials() { return kMseBlocks; }

// ------------------------------------------------------------------------------------------ calibration loop
// Adam (Kingma and Ba 2015, algorithm 1) on (mu, xi) in binary64, one thread: the host loop's arithmetic in
// its order (bias corrections from running products of the rates, the step clamped at the lower bounds), so
// a loop that stays on the device takes the same steps.
__global__ void k_calib_init(RunSpec spec, ::avl_params start, RunSpec* __restrict__ spec_dev,
                             ::avl_params* __restrict__ p_dev, double* __restrict__ st, int32_t* __restrict__ err) {
    *spec_dev = spec;
    *p_dev = start;
    st[0] = (double)start.mu;
    st[1] = (double)start.xi;
    st[2] = st[3] = st[4] = st[5] = 0.0;
    st[6] = st[7] = 1.0;
    err[0] = err[1] = 0;
}

__global__ void k_adam_step(const double* __restrict__ scal, const int32_t* __restrict__ status,
                            double* __restrict__ st, ::avl_params* __restrict__ p, double* __restrict__ row,
                            AdamConsts c, int32_t t, int32_t* __restrict__ err) {
    if (*status != 0 && err[0] == 0) {
        err[0] = *status;
        err[1] = t;
    }
    row[0] = scal[0];
    row[1] = st[0];
    row[2] = st[1];
    row[3] = scal[1];
    row[4] = scal[2];
    st[6] *= c.b1;
    st[7] *= c.b2;
    for (int k = 0; k < 2; ++k) {
        const double g = scal[1 + k];
        st[2 + k] = c.b1 * st[2 + k] + (1.0 - c.b1) * g;
        st[4 + k] = c.b2 * st[4 + k] + (1.0 - c.b2) * (g * g);
        const double mh = st[2 + k] / (1.0 - st[6]);
        const double vh = st[4 + k] / (1.0 - st[7]);
        double th = st[k] - c.lr[k] * mh / (sqrt(vh) + c.eps);
        if (th < c.lo[k]) th = c.lo[k];
        st[k] = th;
    }
    p->mu = (float)st[0];
    p->xi = (float)st[1];
}

hipError_t launch_calib_init(RunSpec spec, ::avl_params start, RunSpec* spec_dev, ::avl_params* p_dev, double* state,
                             int32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_calib_init, dim3(1), dim3(1), 0, s, spec, start, spec_dev, p_dev, state, err);
    return hipGetLastError();
}

hipError_t launch_adam_step(const double* scal, const int32_t* status, double* state, ::avl_params* p_dev,
                            double* row, AdamConsts c, int32_t t, int32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_adam_step, dim3(1), dim3(1), 0, s, scal, status, state, p_dev, row, c, t, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ launchers

size_t smooth_checkpoints(uint32_t S) { return S == 0 ? 0 : (S + kCkpt - 1) / kCkpt; }
size_t smooth_scratch_bytes() { return (size_t)kCkpt * kBackwardGrid * kSmoothBlock * sizeof(float2); }
size_t smooth_reduce_blocks(unsigned long long cap) { return (size_t)((cap + kReduceChunk - 1) / kReduceChunk) + 1; }

namespace {

struct SmoothVariant {
    int block;
    uint32_t spl;
};
// forward candidates: (threads per block, slots per lane); backward: slots per lane at 256 threads
constexpr SmoothVariant kFwdVariants[] = {{256, 8}, {1024, 2}, {512, 2}, {1024, 1}, {256, 2}, {512, 4}};
constexpr uint32_t kBwdSpl[] = {8, 2, 1, 4};

template <int kBlk>
void launch_fwd(const SmoothArgs& a, hipStream_t s) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_smooth_forward<kBlk>),
                                                     kBlk, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    hipLaunchKernelGGL(k_smooth_forward<kBlk>, dim3(cus * per_cu), dim3(kBlk), 0, s, a);
}

}  // namespace

int smooth_forward_variants() { return (int)(sizeof(kFwdVariants) / sizeof(kFwdVariants[0])); }
int smooth_backward_variants() { return (int)(sizeof(kBwdSpl) / sizeof(kBwdSpl[0])); }

hipError_t launch_smooth_forward(const SmoothArgs& a, int variant, hipStream_t s) {
    if (variant < 0 || variant >= smooth_forward_variants()) variant = 0;
    SmoothArgs b = a;
    b.spl = kFwdVariants[variant].spl;
    switch (kFwdVariants[variant].block) {
        case 1024: launch_fwd<1024>(b, s); break;
        case 512: launch_fwd<512>(b, s); break;
        default: launch_fwd<256>(b, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_smooth_backward_kernel(const SmoothArgs& a, int variant, hipStream_t s) {
    if (variant < 0 || variant >= smooth_backward_variants()) variant = 0;
    SmoothArgs b = a;
    b.spl = kBwdSpl[variant];
    hipLaunchKernelGGL(k_smooth_backward, dim3(kBackwardGrid), dim3(kSmoothBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_smooth_reductions(const SmoothArgs& a, const int32_t* n_cells, float* dmass, int64_t n_grid,
                                    double* part, double* dparams, hipStream_t s) {
    const int nb = (int)smooth_reduce_blocks(a.cap);
    hipLaunchKernelGGL(k_reduce_params, dim3(nb), dim3(256), 0, s, a.pp, a.cap, a.runs, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, part, nb, dparams);
    const unsigned blocks = (unsigned)((n_grid + 255) / 256);
    if (blocks) hipLaunchKernelGGL(k_dmass, dim3(blocks), dim3(256), 0, s, a.pp + 3 * a.cap, a.cells, n_cells, a.runs, dmass);
    return hipGetLastError();
}

hipError_t launch_q_to_float(const unsigned long long* q, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_q_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, n, out);
    return hipGetLastError();
}

}  // namespace avl
