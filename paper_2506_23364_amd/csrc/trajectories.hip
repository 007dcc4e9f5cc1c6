// Particle trajectories of the avalanche overlay (section 5.2 of arXiv 2506.23364, the trajectory node):
// particles released per coded texel, steered by persistence and a random deviation from the optimal
// (downslope) path, slowed by Coulomb/Voellmy friction, stopped by the energy line or a runout angle;
// accumulated into a hit-count raster and a max-velocity raster. One kernel serves a single run and a
// batch of runs (parameter sets x DEM tiles x release scenarios) in one persistent launch.
//
// Design for gfx950 (measured choices; the alternatives are recorded in the design notes):
//  - One persistent grid sized to the chip's occupancy; one lane carries one particle at a time and its
//    whole state stays in VGPRs. A lane whose particle ended takes the next particle slot in the same
//    iteration, from a per-wave reservoir refilled 64 slots at a time.
//  - Slots are ordered replica-major within a release cell and run-major across runs; every run starts
//    at a multiple of 64, so a 64-slot chunk belongs to one run. Release cells are in row-major order,
//    so consecutive slots start at the same or neighbouring cells and their paths share most cells.
//  - Device-scope atomics on the rasters are performed beyond L2 (at the memory side), so they are the
//    cost to cut. Entry counts and per-cell max v^2 go first into a table in LDS shared by the whole
//    workgroup (tag, count, max; linear probing), flushed to the rasters at epoch boundaries (a pair of
//    barriers every kFlush iterations per wave on average). A cell whose probes are all held by other
//    cells goes straight to the raster.
//  - An epoch is a budget of kFlush x (waves per block) wave-iterations that the block's waves claim one
//    at a time from an LDS counter, so a wave that runs faster than its neighbours does more of them and
//    every wave reaches the boundary within about one iteration of the others (a fixed count per wave
//    left the fast waves waiting at the first barrier for 15-25 % of their time).
//  - The waves of a workgroup share a window of consecutive slots (two ranges, topped up at epoch
//    boundaries), so the table sees the paths of neighbouring release cells together. Top-ups are guided:
//    up to kWindow x kBlock slots, but at most half the partition's remainder over the blocks of an XCD,
//    so windows shrink as the queues drain and the blocks finish together. A wave that runs the window
//    dry mid-epoch takes 64-slot chunks from the queues directly.
//  - The slot range is split into one partition per XCD; windows and chunks come from the XCD's own
//    partition first and from the others only when it is empty. Each XCD's L2 then holds its own band
//    of the DEM (or its own runs).
//  - Every run writes the caller's rasters directly (v^2 bits, turned into speeds by a finalize pass).
//    Per-XCD private copies bought nothing once the table had cut the atomics: the atomics are
//    performed at the memory side either way, and zeroing and merging the copies cost 9 % at 8192^2.
//  - Accumulation is integer only (u32 add; u32 max on the bits of v^2 >= 0, whose order is the value
//    order), so every raster is independent of scheduling and of the kernel variant: bit-reproducible.
//  - Philox4x32-10 gives four words per block; one block serves two consecutive steps.
#include "particle.h"

namespace avl {

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
using dev::kChunk;

// LDS table accesses are relaxed atomics: lanes of the wave update slots concurrently.
__device__ __forceinline__ uint32_t lds_ld(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A raster cell's v^2 bits as this CU's caches hold them: a workgroup-scope read, served by L1 or the XCD's
// L2 when they hold the line. The raster's maxima are performed at the memory side, so the cached value can
// be older than the memory's, but every value the cell takes during the pass is at least the one before
// it (it is zeroed before the launch, and the kernel's start discards lines cached before that), so a
// read that is already >= v proves a max with v unnecessary. A read from the memory side (nontemporal)
// took 1.27x as long over the 8192^2 pass: each epoch boundary waits for these reads.
__device__ __forceinline__ uint32_t cached_bits(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Max into a global raster cell, skipped when a cached read already shows a value >= bits.
__device__ __forceinline__ void global_max(uint32_t* __restrict__ p, uint32_t bits) {
    if (cached_bits(p) < bits) atomicMax(p, bits);
}

}  // namespace

using namespace dev;

// Workgroup-shared accumulation table: kTbl slots of (cell key, entry count, max v^2 bits) in LDS,
// open addressing with a few linear probes. A particle's visit to a cell (from its entry, or its release,
// to the step that leaves the cell or ends the path) goes into the table once, when it ends: one entry
// and the visit's largest v^2 (the counts are the same as counting each entry when it happens, and one
// table operation per visit replaces a claim at the entry plus a max at the exit). Slots are emptied only
// at epoch boundaries: each boundary flushes a slot to the rasters and empties it, except (with retention
// on) a slot whose cell saw enough visits end in the epoch that ended, which keeps its key, count and
// maximum into the next epoch. With retention the count word holds two 16-bit halves: the entries so far
// (low) and their number at the last boundary (high).
template <int kTbl>
struct Table {
    uint32_t tag[kTbl], cnt[kTbl], vmx[kTbl];
};

// Workgroup control block in LDS. The window is a range of consecutive slots that the workgroup's waves
// share; it changes only between the barriers of an epoch boundary.
struct Control {
    unsigned long long base[2];   // the window: two ranges of consecutive slots, taken in order
    uint32_t len[2];              // their lengths (multiples of 64)
    uint32_t take;                // window slots handed out this epoch (grows by 64 per take)
    uint32_t busy[2];             // waves with work left, per epoch parity
    uint32_t part, tried, empty;  // the window's own walk over the XCD partitions
    uint32_t dry;                 // the tail probe has seen the block run out of slots
    uint32_t iters;               // wave-iterations of the epoch's budget claimed so far
    unsigned long long left;      // slots left in the partition after the window's last top-up
    unsigned long long st[4];     // single run: the block's statistics, summed when its waves are done
};

// kAlpha: the runout-angle stop is compiled in; a single run without it takes the instantiation without.
// A single run with it keeps the release point and height in registers; a batch re-derives them from the
// release cell when a run uses the stop, so its kernel carries no registers for them.
// kKeep: table retention, 0 off; else a slot whose cell saw at least kKeep visits end in the epoch that
// ended stays in the table (its count and maximum reach the rasters at a later boundary).
// kWpe: waves per SIMD the register budget is sized for (8: 64 VGPRs; 6: 80).
// kRec: the recording instantiation (single run): the particles of the recorded range also write their
// points and end records (a diagnostic; the other instantiations compile none of it).
template <bool kBatch, bool kAlpha, int kBlock, int kFlush, int kTbl, int kProbes, int kWindow, int kKeep, int kWpe = 8,
          bool kRec = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWpe)))
void k_trajectories(TrajArgs a) {
    static_assert(!(kRec && kBatch), "recording is for single runs");
    // a lane ends at most one visit per iteration and a block runs at most kFlush x (waves per block)
    // wave-iterations per epoch, so a slot gains at most kBlock * kFlush entries per epoch; a
    // retained count stays below kKeepCap, so the low half never carries
    static_assert(kKeep == 0 || kBlock * kFlush <= 32768, "retention needs 16-bit counts per epoch");
    constexpr uint32_t kKeepCap = 65536u - (uint32_t)(kBlock * kFlush);
    constexpr uint32_t kSuper = (uint32_t)kWindow * kBlock;  // slots per window top-up
    static_assert(kTbl % kBlock == 0, "every thread flushes the same number of table slots");
    constexpr int kPer = kTbl / kBlock;
    __shared__ Table<kTbl> tb;
    __shared__ Control ctl;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint64_t total = wave_bcast64(a.run_off[a.n_runs]);
    // A small problem runs on fewer blocks: with ~1 particle per lane every wave would issue the whole
    // iteration for a few live lanes, and the waves of a SIMD would share its issue slots until the
    // longest path ends. Blocks past what gives each lane about the variant's slots per lane leave at once.
    if ((uint64_t)blockIdx.x >= active_blocks(total, kBlock, a.slots_per_lane)) return;
    const int W = a.W, H = a.H;
    const float fW = (float)W, fH = (float)H;
    const uint32_t xcd = xcd_id();
    uint32_t* const counts = a.counts;
    uint32_t* const vmax2 = a.vmax2;
    const uint32_t Wp = (uint32_t)W + 2u, row_bytes = 4u * Wp;  // rows of the padded DEM tiles

    for (int k = threadIdx.x; k < kTbl; k += kBlock) {
        tb.tag[k] = kEmpty;
        tb.cnt[k] = 0u;
        tb.vmx[k] = 0u;
    }

    // Takes up to `len` consecutive slots from the XCD queues, starting with this XCD's partition and
    // moving on when it is empty; [base, end) is empty once every partition is. Single lane.
    // `left` receives what remained of the partition after the take.
    auto take_global = [&](uint32_t& part, uint32_t& tried, uint32_t& empty, uint32_t len, uint64_t& base,
                           uint64_t& end, uint64_t& left) {
        base = end = left = 0;
        while (!empty) {
            const uint64_t pb = part_begin(total, part), pe = part_begin(total, part + 1);
            const uint64_t got = atomicAdd(a.queues + part * kQueueStride, (unsigned long long)len);
            if (pb + got < pe) {
                base = pb + got;
                end = (base + len < pe) ? base + len : pe;
                left = pe - end;
                return;
            }
            part = (part + 1) % kXcds;
            if (++tried >= (uint32_t)kXcds) empty = 1u;
        }
    };

    // table slot of `key`, claimed if a probe finds an empty slot first; -1 if every probe is held by
    // another cell. Within an epoch slots are only filled, never emptied, so a key's first probe that is
    // empty or holds it is the same for every lane. (A retained key can find an earlier probe emptied at
    // the boundary and take that one as well: two slots of one cell, both flushed, the sums unchanged.)
    // The probes' tags are read in groups of kGroup, one LDS round trip per group, and the group's slots
    // are then taken in probe order: a read that shows the key is final (only the key's own claim writes
    // it), one that shows another key stays true (slots are not emptied within an epoch), and one that shows
    // an empty slot is settled by the compare-and-swap. So the slot taken is the first in probe order that
    // is empty or holds the key, as with one probe at a time, but a claim no longer waits for up to kProbes
    // dependent round trips.
    auto claim = [&](uint32_t key) -> int {
        constexpr int kGroup = 4;
        const uint32_t h = (uint32_t)(((uint64_t)(key * 0x9E3779B1u) * (uint64_t)kTbl) >> 32);
#pragma unroll
        for (int g = 0; g < kProbes; g += kGroup) {
            uint32_t sl[kGroup], t[kGroup];
#pragma unroll
            for (int i = 0; i < kGroup && g + i < kProbes; ++i) {
                sl[i] = h + (uint32_t)(g + i);
                if (sl[i] >= (uint32_t)kTbl) sl[i] -= (uint32_t)kTbl;
                t[i] = lds_ld(tb.tag + sl[i]);
            }
#pragma unroll
            for (int i = 0; i < kGroup && g + i < kProbes; ++i) {
                uint32_t ti = t[i];
                if (ti == kEmpty) {
                    const uint32_t old = atomicCAS(tb.tag + sl[i], kEmpty, key);
                    ti = (old == kEmpty) ? key : old;
                }
                if (ti == key) return (int)sl[i];
            }
        }
        return -1;
    };

    // Shifts the window past the slots handed out in the epoch that ended and tops it up with a new
    // range when the second range has been reached. Thread 0, between the barriers of a boundary.
    const uint64_t guide_div = 2ull * max(1u, gridDim.x / (uint32_t)kXcds);  // 2 x blocks per XCD
    auto refill_window = [&](bool first) {
        if (first) {
            ctl.base[0] = ctl.base[1] = 0;
            ctl.len[0] = ctl.len[1] = 0;
            ctl.take = 0;
            ctl.busy[0] = ctl.busy[1] = 0;
            ctl.part = xcd;
            ctl.tried = 0;
            ctl.empty = total == 0 ? 1u : 0u;
            ctl.left = ~0ull;
            ctl.dry = 0u;
            ctl.iters = 0u;
        }
        const uint32_t l0 = ctl.len[0], l1 = ctl.len[1];
        const uint32_t t = min(ctl.take, l0 + l1);
        if (t >= l0) {
            ctl.base[0] = ctl.base[1] + (t - l0);
            ctl.len[0] = l1 - (t - l0);
            ctl.base[1] = 0;
            ctl.len[1] = 0;
        } else {
            ctl.base[0] += t;
            ctl.len[0] = l0 - t;
        }
        ctl.take = 0;
        if (ctl.len[1] == 0u) {
            // guided top-up: a share of what the partition had left, so windows shrink as the queues
            // drain and every block runs out of work at about the same time
            const uint64_t share = ctl.left / guide_div;
            const uint32_t want = share >= kSuper ? kSuper : max(kChunk, (uint32_t)share & ~(kChunk - 1u));
            uint64_t wb = 0, we = 0, left = 0;
            take_global(ctl.part, ctl.tried, ctl.empty, want, wb, we, left);
            ctl.base[1] = wb;
            ctl.len[1] = (uint32_t)(we - wb);
            ctl.left = left;
        }
    };
    // tail probe (diagnostics): per block the real-time clock at its start, when it first finds no slot left
    // in its window nor in any queue, and at its end
    unsigned long long* const probe = a.probe ? a.probe + 3 * (size_t)blockIdx.x : nullptr;
    if (threadIdx.x == 0) {
        if (probe) probe[0] = __builtin_amdgcn_s_memrealtime();
        refill_window(true);
    }
    __syncthreads();

    // The wave's run: its constants in scalar registers and its padded DEM tile through a buffer
    // resource (32-bit offsets, no clamps). A single run keeps run 0; in a batch a wave works on one run
    // at a time, and slots of the next run wait in its reservoir until the wave has no particle left.
    uint32_t wrun = 0;
    RunConst rc = uniform_run(a.runs[0]);
    __amdgpu_buffer_rsrc_t dem_rs = buffer_rsrc(a.dem_pad + rc.pad_off, a.pad_bytes);

    // per-lane statistics of run wrun, added to the run's counters when the wave changes run or ends. A
    // step is a move that does not hit the step limit: it is accepted, leaves the grid or stops, so the
    // steps are the accepted ones (each particle's final n, added when its lane takes the next particle or
    // the statistics are flushed) plus the exits and stops, and no counter moves per step for them.
    uint64_t st_acc = 0;
    uint32_t st_exit = 0, st_stop = 0, st_limit = 0;
    uint32_t n = 0;  // the lane's particle: accepted steps so far (not yet in st_acc)
    auto flush_stats = [&]() {
        st_acc += n;
        n = 0;
        const uint64_t s1 = wave_sum64(st_exit), s2 = wave_sum64(st_stop);
        const uint64_t s0 = wave_sum64(st_acc) + s1 + s2, s3 = wave_sum64(st_limit);
        if (lane == 0) {
            unsigned long long* st = a.stats + 4 * (size_t)wrun;
            if (s0) atomicAdd(st + 0, (unsigned long long)s0);
            if (s1) atomicAdd(st + 1, (unsigned long long)s1);
            if (s2) atomicAdd(st + 2, (unsigned long long)s2);
            if (s3) atomicAdd(st + 3, (unsigned long long)s3);
        }
        st_acc = 0;
        st_exit = st_stop = st_limit = 0;
    };

    // wave-uniform slot state: this wave's own walk over the XCD partitions (once the window is spent),
    // and a reservoir of up to 64 slots with the run they belong to
    uint32_t part = xcd, tried = 0, queue_empty = (total == 0) ? 1u : 0u;
    uint64_t res_next = 0, res_end = 0;
    uint32_t res_run = 0;

    // lane state
    bool alive = false;
    float x = 0, y = 0, z = 0, gx = 0, gy = 0, dx = 0, dy = 0, v2 = 0, x0 = 0, y0 = 0, zr = 0, cmax2 = 0;
    uint32_t rep = 0, cell_id = 0, spare_x = 0, spare_y = 0, cur = 0;
    uint32_t rk = ~0u;  // recording: index of the lane's particle in the recorded range, ~0 if outside it
    auto rec_point = [&](uint32_t m, float px, float py, float pv2) {
        if constexpr (kRec) {
            if (rk == ~0u || !a.rec_xy) return;
            unsigned long long at;
            if (a.rec_off) {
                at = a.rec_off[rk] + m;
            } else {
                if (m >= a.rec_stride) return;
                at = (unsigned long long)rk * a.rec_stride + m;
            }
            a.rec_xy[at] = make_float2(px, py);
            if (a.rec_v2) a.rec_v2[at] = pv2;
        }
    };
    auto rec_end = [&](uint32_t why) {
        if constexpr (kRec) {
            if (rk != ~0u) a.rec_end[rk] = (n << 2) | why;
        }
    };


    constexpr uint32_t kBudget = (uint32_t)kFlush * (uint32_t)(kBlock / kWave);  // wave-iterations per epoch
    uint32_t wit = 0;  // the wave's iterations so far; a live particle's step count has their parity
    for (uint32_t epoch = 0;; ++epoch) {
        // the window of this epoch
        const uint64_t wb0 = wave_bcast64(ctl.base[0]), wb1 = wave_bcast64(ctl.base[1]);
        const uint32_t wl0 = uniform_u(ctl.len[0]), wl1 = uniform_u(ctl.len[1]);
        bool win_out = wl0 + wl1 == 0u;
        bool finished = false;

        // the wave claims each iteration of the epoch's budget one iteration ahead, so the LDS round trip
        // overlaps the iteration before it
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(&ctl.iters, 1u);
        for (;;) {
            const uint64_t idle = __ballot(!alive);
            const int nidle = __popcll(idle);
            const bool drained = win_out && queue_empty && res_next >= res_end;
            if (nidle == kWave && drained) {
                finished = true;
                break;
            }
            if (__builtin_amdgcn_readfirstlane(ticket) >= kBudget) break;
            const uint32_t it = wit++;
            if (lane == 0) ticket = atomicAdd(&ctl.iters, 1u);

            // ---- hand slots to idle lanes in lane order: the reservoir, refilled with the next 64-slot
            // chunk of the window (else of the queues) when it runs dry. Only on the wave's even iterations:
            // every particle then starts on an even iteration, so its step parity is the iteration's and
            // the Philox block (one per two steps) is a uniform branch.
            bool fresh = false;
            if ((it & 1) == 0 && nidle > 0 && !drained) {
                // next 64-slot chunk of the window, else of the queues; empty when neither has any left
                auto next_chunk = [&](uint64_t& base, uint64_t& cend) {
                    base = cend = 0;
                    if (!win_out) {
                        uint32_t v = 0;
                        if (lane == 0) v = atomicAdd(&ctl.take, kChunk);
                        v = __builtin_amdgcn_readfirstlane(v);
                        // the ranges are multiples of 64 long, so a chunk never straddles them
                        if (v < wl0) {
                            base = wb0 + v;
                            cend = base + min(wl0 - v, kChunk);
                        } else if (v - wl0 < wl1) {
                            base = wb1 + (v - wl0);
                            cend = base + min(wl1 - (v - wl0), kChunk);
                        } else {
                            win_out = true;
                        }
                    }
                    if (cend == base && !queue_empty) {
                        uint64_t gb = 0, ge = 0, gl = 0;
                        if (lane == 0) take_global(part, tried, queue_empty, kChunk, gb, ge, gl);
                        base = wave_bcast64(gb);
                        cend = wave_bcast64(ge);
                        queue_empty = __builtin_amdgcn_readfirstlane(queue_empty);
                        part = __builtin_amdgcn_readfirstlane(part);
                        tried = __builtin_amdgcn_readfirstlane(tried);
                    }
                };
                const int rank = __popcll(idle & below);
                uint64_t slot = ~0ull;
                if constexpr (!kBatch) {
                    // one run: the reservoir's remainder, then a new chunk, in one pass
                    const uint64_t avail = res_end - res_next;
                    if (avail >= (uint64_t)nidle) {
                        slot = res_next + rank;
                        res_next += nidle;
                    } else {
                        uint64_t base, cend;
                        next_chunk(base, cend);
                        if ((uint64_t)rank < avail)
                            slot = res_next + rank;
                        else if (base + (rank - avail) < cend)
                            slot = base + (rank - avail);
                        const uint64_t next = base + ((uint64_t)nidle - avail);
                        res_next = next < cend ? next : cend;
                        res_end = cend;
                    }
                } else {
                    // a batch: the same two sources, but a chunk of another run waits in the reservoir
                    // until the wave has no particle of its current run left
                    uint64_t want = idle;  // idle lanes not yet served
#pragma unroll 1
                    for (int round = 0; round < 2 && want != 0ull; ++round) {
                        if (res_next >= res_end) {
                            uint64_t base, cend;
                            next_chunk(base, cend);
                            if (cend == base) break;  // nothing left for this wave
                            res_next = base;
                            res_end = cend;
                            res_run = find_run(a.run_off, a.n_runs, base);
                        }
                        if (res_run != wrun) {
                            if (want != idle || __ballot(alive) != 0ull) break;
                            flush_stats();
                            wrun = res_run;
                            rc = uniform_run(a.runs[wrun]);
                            dem_rs = buffer_rsrc(a.dem_pad + rc.pad_off, a.pad_bytes);
                        }
                        const uint64_t avail = res_end - res_next;
                        const bool mine = ((want >> lane) & 1ull) != 0ull;
                        const int r = __popcll(want & below);
                        const bool served = mine && (uint64_t)r < avail;
                        if (served) slot = res_next + (uint64_t)r;
                        const uint64_t n_want = (uint64_t)__popcll(want);
                        res_next += avail < n_want ? avail : n_want;
                        want &= ~__ballot(served);
                    }
                }
                uint64_t i = 0;  // release-cell index of the new particle within its run
                if (!alive && slot < total) {
                    const uint64_t local = slot - (kBatch ? a.run_off[wrun] : 0ull);
                    if (local < rc.n_slots) {  // past n_slots: padding up to the next multiple of 64
                        i = (local >> 32) == 0 ? (uint64_t)udiv((uint32_t)local, a.pdiv) : local / rc.P;
                        rep = (uint32_t)local - (uint32_t)i * rc.P;
                        fresh = true;
                    }
                }
                if (fresh) {
                    // a single run reads the start state from its per-cell records, and so does a batch run
                    // whose scenario's records were made on its tile (a uniform branch); any other batch run
                    // computes it from the same padded tile the steps read
                    const StartRec st = !kBatch     ? a.starts[i]
                                        : rc.use_rec ? a.starts[rc.cells_off + i]
                                                     : start_state_pad(dem_rs, Wp, row_bytes, W,
                                                                       (uint32_t)a.cells[rc.cells_off + i]);
                    cell_id = st.cell;
                    x = st.x;
                    y = st.y;
                    z = st.z;
                    gx = st.gx;
                    gy = st.gy;
                    dx = st.dx;
                    dy = st.dy;
                    if (kAlpha && !kBatch) {
                        x0 = x;
                        y0 = y;
                        zr = z;
                    }
                    v2 = 0.0f;
                    cmax2 = 0.0f;
                    st_acc += n;  // the lane's previous particle
                    n = 0;
                    // the raster cell of the release point: the release texel's index keys the random
                    // stream, the DEM cell under its centre takes the counts (the same cell at one texel per
                    // DEM cell)
                    cur = rc.raster_off +
                          (kBatch ? cell_id : (uint32_t)(int)floorf(y) * (uint32_t)W + (uint32_t)(int)floorf(x));
                    alive = true;
                    if constexpr (kRec) {
                        const uint64_t k = (uint64_t)i * rc.P + rep;  // the particle's index in the run
                        rk = (k >= a.rec_first && k - a.rec_first < a.rec_n) ? (uint32_t)(k - a.rec_first) : ~0u;
                        rec_point(0u, x, y, 0.0f);
                    }
                }
            }

            // ---- one step of every live particle
            const RunConst& R = rc;
            bool leave = false;  // a visit ended: its cell and largest v^2
            uint32_t leave_bits = 0;
            uint32_t leave_key = 0;
            if (alive) {
                // Every live lane runs the whole step and the outcome selects what it keeps: a lane at the
                // step limit, leaving the grid or stopping discards its target (an off-grid target's gather
                // reads through the buffer's bounds check, so it cannot fault). Without the nested branches
                // the compiler no longer copies the particle state at every join (5 % of the alpine pass).
                const bool lim = n >= a.S;
                uint32_t ux, uy;
                if ((it & 1) == 0) {  // n is even
                    // the key is wave-uniform: pinning it to scalar registers here makes the round keys
                    // scalar adds inside the block instead of 20 loop-invariant values hoisted out of the
                    // loop, spilled to vector lanes and read back by VALU instructions
                    uint32_t k0 = __builtin_amdgcn_readfirstlane(R.key0);
                    uint32_t k1 = __builtin_amdgcn_readfirstlane(R.key1);
                    asm volatile("" : "+s"(k0), "+s"(k1));
                    const uint4 o = philox4x32_10(n >> 1, rep, cell_id, R.run, k0, k1);
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
                // Q = 1 - persistence is 0 or in [2^-24, 1] (persistence in [0, 1])
                const float t = gg > 0.0f ? div_sqrt_rn(R.Q, gg) : 0.0f;
                const float wx = (R.per * dx - t * gx) + R.rnd * rx;
                const float wy = (R.per * dy - t * gy) + R.rnd * ry;
                const float ww = wx * wx + wy * wy;
                if (ww > 0.0f) {
                    const float inv = div_sqrt_rn(1.0f, ww);
                    dx = wx * inv;
                    dy = wy * inv;
                }
                const float x1 = x + R.L * dx;
                const float y1 = y + R.L * dy;
                const float fc1 = floorf(x1), fr1 = floorf(y1);
                const bool inb = !lim && fc1 >= 0.0f && fc1 < fW && fr1 >= 0.0f && fr1 < fH;
                const Sample s1 = bilinear_pad(dem_rs, Wp, row_bytes, x1, y1);
                const float dz = z - s1.z;
                // dl2 + dz^2 >= dl2: with dl2 >= 2^-96 (a run constant) no lane needs the small-argument check
                float ds;
                if (R.dl2 >= 0x1p-96f)
                    ds = sqrt_rn_big(R.dl2 + dz * dz);
                else
                    ds = sqrt_rn(R.dl2 + dz * dz);
                const float num = v2 + a.g2 * (dz - R.mdl);
                bool stop = !(num > 0.0f);
                const float v2n = num / (1.0f + R.cd * ds);
                if (kAlpha && R.use_alpha) {
                    float ax0 = x0, ay0 = y0, azr = zr;
                    if (kBatch) {  // the release cell's centre and the height sampled there
                        const uint32_t rr = udiv(cell_id, a.wdiv), cc = cell_id - rr * (uint32_t)W;
                        ax0 = (float)cc + 0.5f;
                        ay0 = (float)rr + 0.5f;
                        azr = bilinear_pad(dem_rs, Wp, row_bytes, ax0, ay0).z;
                    }
                    const float hx = x1 - ax0, hy = y1 - ay0;
                    stop = stop || (azr - s1.z) < R.tca * sqrtf(hx * hx + hy * hy);
                }
                const bool acc = inb && !stop;
                st_limit += lim ? 1u : 0u;
                st_exit += (!lim && !inb) ? 1u : 0u;
                st_stop += (inb && stop) ? 1u : 0u;
                if constexpr (kRec) {
                    if (lim)
                        rec_end(0u);
                    else if (!inb)
                        rec_end(1u);
                    else if (stop) {
                        rec_point(n + 1u, x1, y1, 0.0f);
                        rec_end(2u);
                    }
                }
                x = acc ? x1 : x;
                y = acc ? y1 : y;
                z = acc ? s1.z : z;
                gx = acc ? s1.gx : gx;
                gy = acc ? s1.gy : gy;
                v2 = acc ? v2n : v2;
                n += acc ? 1u : 0u;
                if constexpr (kRec) {
                    if (acc) rec_point(n, x, y, v2);
                }
                // row x W as a 24-bit multiply (full rate; a 32-bit one is quarter rate): both factors are below
                // 2^23 on an accepted grid and nc is used only for a step inside it
                const uint32_t nc = R.raster_off + __umul24((uint32_t)(int)fr1, (uint32_t)W) + (uint32_t)(int)fc1;
                const bool change = acc && nc != cur;
                leave = change || !acc;
                leave_bits = __float_as_uint(cmax2);
                leave_key = cur;
                cur = change ? nc : cur;
                cmax2 = change ? v2 : ((acc && v2 > cmax2) ? v2 : cmax2);
                alive = acc;
            }
            // ---- accumulate the visit that ended: its entry and its largest v^2 (0 bits: nothing to max)
            if (leave) {
                const int sl = claim(leave_key);
                if (sl >= 0) {
                    atomicAdd(tb.cnt + sl, 1u);
                    if (leave_bits) atomicMax(tb.vmx + sl, leave_bits);
                } else {
                    atomicAdd(counts + leave_key, 1u);
                    if (leave_bits) global_max(vmax2 + leave_key, leave_bits);
                }
            }
        }

        // ---- epoch boundary: count the waves with work left, flush the table, refill the window
        if (lane == 0 && !finished) atomicAdd(&ctl.busy[epoch & 1u], 1u);
        __syncthreads();
        if (threadIdx.x == 0) {
            ctl.busy[(epoch + 1) & 1u] = 0u;
            ctl.iters = 0u;
            refill_window(false);
            if (probe && !ctl.dry && ctl.empty && ctl.len[0] == 0u) {
                ctl.dry = 1u;
                probe[1] = __builtin_amdgcn_s_memrealtime();
            }
        }
        // flush this thread's kPer slots: all raster reads of the max check are issued before any is
        // used, so the flush costs one memory round trip rather than one per slot. The last boundary
        // (no wave has work left) flushes every slot.
        const bool last = ctl.busy[epoch & 1u] == 0u;
        uint32_t ft[kPer], fc[kPer], fv[kPer], fg[kPer];
        bool keep[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = threadIdx.x + j * kBlock;
            ft[j] = tb.tag[k];
            fc[j] = tb.cnt[k];
            fv[j] = tb.vmx[k];
            if constexpr (kKeep > 0) {
                const uint32_t c = fc[j] & 0xFFFFu, seen = fc[j] >> 16;
                keep[j] = !last && ft[j] != kEmpty && c - seen >= (uint32_t)kKeep && c < kKeepCap;
                fc[j] = c;
            } else {
                keep[j] = false;
            }
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j)  // an empty slot reads cell 0: no branch between the loads
            fg[j] = keep[j] ? 0u : cached_bits(vmax2 + (ft[j] != kEmpty ? ft[j] : 0u));
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = threadIdx.x + j * kBlock;
            if (keep[j]) {
                tb.cnt[k] = fc[j] | (fc[j] << 16);
            } else if (ft[j] != kEmpty) {
                if (fc[j]) atomicAdd(counts + ft[j], fc[j]);
                tb.tag[k] = kEmpty;
                tb.cnt[k] = 0u;
                tb.vmx[k] = 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j)  // a stale read >= v suffices
            if (!keep[j] && ft[j] != kEmpty && fg[j] < fv[j]) atomicMax(vmax2 + ft[j], fv[j]);
        __syncthreads();
        if (ctl.busy[epoch & 1u] == 0u) break;
    }
    if constexpr (kBatch) {
        flush_stats();
    } else {
        // every wave leaves the loop at the same boundary: the block's statistics are summed in LDS and
        // reach the four counters with one atomic each per block, not per wave (the counters share a
        // memory line, where device-scope atomics serialise)
        unsigned long long* const bst = ctl.st;
        if (threadIdx.x < 4) bst[threadIdx.x] = 0ull;
        __syncthreads();
        st_acc += n;
        const uint64_t s1 = wave_sum64(st_exit), s2 = wave_sum64(st_stop);
        const uint64_t s0 = wave_sum64(st_acc) + s1 + s2, s3 = wave_sum64(st_limit);
        if (lane == 0) {
            if (s0) atomicAdd(bst + 0, (unsigned long long)s0);
            if (s1) atomicAdd(bst + 1, (unsigned long long)s1);
            if (s2) atomicAdd(bst + 2, (unsigned long long)s2);
            if (s3) atomicAdd(bst + 3, (unsigned long long)s3);
        }
        __syncthreads();
        if (threadIdx.x < 4 && bst[threadIdx.x]) atomicAdd(a.stats + threadIdx.x, bst[threadIdx.x]);
    }
    if (probe && threadIdx.x == 0) probe[2] = __builtin_amdgcn_s_memrealtime();
}

// ------------------------------------------------------------------------------------------ start records

__global__ __launch_bounds__(256) void k_start_records(const float* __restrict__ dem, int H, int W, uint32_t mult,
                                                       const int32_t* __restrict__ cells,
                                                       const int32_t* __restrict__ n_cells, int64_t cap,
                                                       StartRec* __restrict__ starts) {
    const int64_t n = min((int64_t)*n_cells, cap);  // records of the first `cap` cells at most
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        starts[i] = start_state(dem, H, W, mult, (uint32_t)cells[i]);
}

hipError_t launch_start_records(const float* dem, int H, int W, int mult, const int32_t* cells,
                                const int32_t* n_cells, int64_t n, StartRec* starts, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_start_records, dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)), dim3(256),
                       0, s, dem, H, W, (uint32_t)mult, cells, n_cells, n, starts);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ run table

// One block: per run, derived constants and slot counts, then the exclusive scan of the padded slot
// counts. A run with an index out of range or invalid parameters gets no slots and status != 0.
__global__ __launch_bounds__(1024) void k_setup_runs(const RunSpec* __restrict__ specs,
                                                     const ::avl_params* __restrict__ params, uint32_t n_params,
                                                     RunSpec one_spec, ::avl_params one_param,
                                                     const int32_t* __restrict__ n_cells_per_scen, uint32_t n_scen,
                                                     uint32_t n_tiles, uint32_t n_runs, int32_t H, int32_t W,
                                                     float cs, uint32_t P, int32_t batched,
                                                     RunConst* __restrict__ runs,
                                                     unsigned long long* __restrict__ run_off,
                                                     int32_t* __restrict__ status, int64_t cap_cells,
                                                     int32_t* __restrict__ rec_run) {
    __shared__ unsigned long long wsum[1024 / kWave];
    const uint32_t per_thread = (n_runs + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per_thread;
    const uint64_t HW = (uint64_t)H * W;
    unsigned long long local = 0;
    for (uint32_t k = 0; k < per_thread; ++k) {
        const uint32_t r = b0 + k;
        if (r >= n_runs) break;
        const RunSpec sp = specs ? specs[r] : one_spec;
        int32_t bad = 0;
        if (sp.tile >= n_tiles || sp.scenario >= n_scen || (specs && sp.param >= n_params)) bad = 1;
        ::avl_params p = one_param;
        if (!bad && specs) p = params[sp.param];
        if (!bad) {
            const bool ok = __builtin_isfinite(p.mu) && p.mu >= 0.0f && !__builtin_isnan(p.xi) && p.xi > 0.0f &&
                            __builtin_isfinite(p.flow_height) && p.flow_height > 0.0f && p.persistence >= 0.0f &&
                            p.persistence <= 1.0f && __builtin_isfinite(p.randomness) && p.randomness >= 0.0f &&
                            __builtin_isfinite(p.step_cells) && p.step_cells > 0.0f && p.step_cells <= 16.0f &&
                            __builtin_isfinite(p.tan_alpha) && p.flags == 0u;
            if (!ok) bad = 2;
        }
        if (!bad && cap_cells >= 0 && (int64_t)n_cells_per_scen[sp.scenario] > cap_cells) bad = 3;
        RunConst c{};
        // derived constants, binary32, in this order
        const float g = 9.81f;
        const float g2 = g + g;
        c.per = p.persistence;
        c.Q = 1.0f - c.per;
        c.rnd = p.randomness;
        c.L = p.step_cells;
        const float dl = c.L * cs;
        c.dl2 = dl * dl;
        c.mdl = p.mu * dl;
        c.cd = g2 / (p.xi * p.flow_height);
        c.use_alpha = p.tan_alpha >= 0.0f ? 1u : 0u;
        c.tca = p.tan_alpha * cs;
        c.key0 = (uint32_t)sp.seed;
        c.key1 = (uint32_t)(sp.seed >> 32);
        c.run = sp.run_id;
        c.dem_off = (uint32_t)(sp.tile * HW);
        c.pad_off = (uint32_t)(sp.tile * (uint64_t)padded_cells(H, W));
        c.cells_off = (uint32_t)(sp.scenario * HW);
        c.raster_off = batched ? (uint32_t)(r * HW) : 0u;
        c.P = P;
        c.n_slots = bad ? 0ull : (unsigned long long)(uint32_t)n_cells_per_scen[sp.scenario] * P;
        runs[r] = c;
        if (status) status[r] = bad;
        if (!bad && rec_run) atomicMin(rec_run + sp.scenario, (int32_t)r);
        local += (c.n_slots + kChunk - 1) / kChunk * kChunk;
    }
    // exclusive scan of the per-thread sums
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    unsigned long long inc = local;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long t = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += t;
    }
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
    for (int k = 0; k < 1024 / kWave; ++k) {
        before += (k < wid) ? wsum[k] : 0ull;
        tot += wsum[k];
    }
    unsigned long long run = before + inc - local;
    for (uint32_t k = 0; k < per_thread; ++k) {
        const uint32_t r = b0 + k;
        if (r >= n_runs) break;
        run_off[r] = run;
        run += (runs[r].n_slots + kChunk - 1) / kChunk * kChunk;
        // every run's atomicMin has completed at the barrier above; read the result past the L1
        if (rec_run && specs && specs[r].scenario < n_scen && specs[r].tile < n_tiles) {
            const int32_t first =
                __hip_atomic_load(rec_run + specs[r].scenario, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            runs[r].use_rec = (first != 0x7FFFFFFF && specs[first].tile == specs[r].tile) ? 1u : 0u;
        }
    }
    if (threadIdx.x == 0) run_off[n_runs] = tot;
}

hipError_t launch_setup_runs(const RunSpec* specs, const ::avl_params* params, uint32_t n_params, RunSpec one_spec,
                             ::avl_params one_param, const int32_t* n_cells_per_scen, uint32_t n_scen, uint32_t n_tiles,
                             uint32_t n_runs, int32_t H, int32_t W, float cell_size, uint32_t P, bool batched,
                             RunConst* runs, unsigned long long* run_off, int32_t* status, hipStream_t s,
                             int64_t cap_cells, int32_t* rec_run) {
    hipLaunchKernelGGL(k_setup_runs, dim3(1), dim3(1024), 0, s, specs, params, n_params, one_spec, one_param,
                       n_cells_per_scen, n_scen, n_tiles, n_runs, H, W, cell_size, P, batched ? 1 : 0, runs, run_off,
                       status, cap_cells, rec_run);
    return hipGetLastError();
}

// Batch start records: scenario s's cells on the tile of its first valid run, from the padded tile (the
// same values the trajectory kernel would read, so the same start states).
__global__ __launch_bounds__(256) void k_batch_records(const RunSpec* __restrict__ specs,
                                                       const int32_t* __restrict__ rec_run,
                                                       const int32_t* __restrict__ n_cells_per_scen, uint32_t n_scen,
                                                       const int32_t* __restrict__ cells, const float* dem_pad, int H,
                                                       int W, StartRec* __restrict__ starts) {
    const uint64_t HW = (uint64_t)H * W;
    const uint32_t Wp = (uint32_t)W + 2u, row_bytes = 4u * Wp;
    const uint64_t np = (uint64_t)padded_cells(H, W);
    for (uint32_t sc = blockIdx.y; sc < n_scen; sc += gridDim.y) {
        const int32_t first = rec_run[sc];
        if (first == 0x7FFFFFFF) continue;  // no valid run uses this scenario
        const __amdgpu_buffer_rsrc_t rs =
            buffer_rsrc(dem_pad + (uint64_t)specs[first].tile * np, (uint32_t)(np * sizeof(float)));
        const int64_t nc = n_cells_per_scen[sc];
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x)
            starts[sc * HW + i] = start_state_pad(rs, Wp, row_bytes, W, (uint32_t)cells[sc * HW + i]);
    }
}

hipError_t launch_batch_records(const RunSpec* specs, const int32_t* rec_run, const int32_t* n_cells_per_scen,
                                uint32_t n_scen, const int32_t* cells, const float* dem_pad, int32_t H, int32_t W,
                                StartRec* starts, hipStream_t s) {
    const uint32_t gy = n_scen < 1024u ? n_scen : 1024u;
    hipLaunchKernelGGL(k_batch_records, dim3(64, gy), dim3(256), 0, s, specs, rec_run, n_cells_per_scen, n_scen, cells,
                       dem_pad, H, W, starts);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ variants

namespace {

struct Variant {
    const void* single;
    const void* batch;
    int block;
    uint32_t spl;  // particle slots per lane that size the grid of a small problem
    int shape[7];  // block, iterations per epoch, table slots, probes, window, retention, waves per SIMD
    void (*launch_single)(dim3, dim3, hipStream_t, const TrajArgs&);        // runout-angle stop compiled in
    void (*launch_single_plain)(dim3, dim3, hipStream_t, const TrajArgs&);  // without it
    void (*launch_batch)(dim3, dim3, hipStream_t, const TrajArgs&);
};

template <bool B, bool A, int Blk, int F, int T, int Q, int M, int K, int Wpe>
void launch_t(dim3 g, dim3 t, hipStream_t s, const TrajArgs& a) {
    hipLaunchKernelGGL((k_trajectories<B, A, Blk, F, T, Q, M, K, Wpe>), g, t, 0, s, a);
}

template <int Blk, int F, int T, int Q, int M, int K, int Wpe = 8>
constexpr Variant make_variant(uint32_t spl = (uint32_t)kSlotsPerLane) {
    return Variant{reinterpret_cast<const void*>(&k_trajectories<false, true, Blk, F, T, Q, M, K, Wpe>),
                   reinterpret_cast<const void*>(&k_trajectories<true, true, Blk, F, T, Q, M, K, Wpe>), Blk, spl,
                   {Blk, F, T, Q, M, K, Wpe},
                   &launch_t<false, true, Blk, F, T, Q, M, K, Wpe>, &launch_t<false, false, Blk, F, T, Q, M, K, Wpe>,
                   &launch_t<true, true, Blk, F, T, Q, M, K, Wpe>};
}

// candidates of the autotuner: (threads per block, iterations per epoch, table slots per block, probes,
// window top-up in blocks of slots, retention threshold[, waves per SIMD of the register budget]) and the
// slots per lane that size a small problem's grid. 1024-thread blocks run two per CU at eight waves per SIMD
// (64 VGPRs; 6144 slots of 12 bytes are 72 KiB of LDS per block); the 768- and 512-thread shapes run at six
// (80 VGPRs), two and three blocks per CU, and the 384-thread shape at six with four blocks per CU. The fifth
// keeps no slot across epochs.
const Variant kVariants[] = {
    make_variant<1024, 16, 6144, 4, 4, 1>(),    make_variant<1024, 32, 6144, 4, 4, 2>(),
    make_variant<1024, 16, 6144, 4, 4, 2>(),    make_variant<1024, 32, 6144, 6, 4, 2>(),
    make_variant<1024, 32, 4096, 4, 4, 0>(),    make_variant<1024, 16, 6144, 8, 4, 2>(),
    make_variant<768, 16, 6144, 8, 4, 2, 6>(),  make_variant<512, 16, 4096, 8, 4, 2, 6>(),
    make_variant<1024, 16, 6144, 4, 4, 1>(2u),  make_variant<1024, 16, 6144, 4, 4, 1>(4u),
    make_variant<1024, 16, 6144, 4, 4, 1>(16u), make_variant<512, 32, 4096, 8, 4, 2, 6>(),
    make_variant<512, 16, 4096, 8, 4, 1, 6>(),  make_variant<768, 16, 6144, 4, 4, 1, 6>(),
    make_variant<384, 16, 3072, 8, 4, 2, 6>(),
};

}  // namespace

int trajectory_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

bool trajectory_variant_info(int variant, int32_t* info) {
    if (variant < 0 || variant >= trajectory_variants()) return false;
    const Variant& v = kVariants[variant];
    for (int i = 0; i < 7; ++i) info[i] = v.shape[i];
    info[7] = (int32_t)v.spl;
    return true;
}

LaunchShape trajectory_shape(bool batched, int variant) {
    if (variant < 0 || variant >= trajectory_variants()) variant = 0;
    const Variant& v = kVariants[variant];
    LaunchShape sh{v.block, 2048, variant};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return sh;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return sh;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched ? v.batch : v.single, v.block, 0) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    sh.grid = cus * per_cu;
    return sh;
}

hipError_t launch_trajectories_record(const TrajArgs& a, hipStream_t s) {
    auto* k = &k_trajectories<false, true, 1024, 16, 6144, 4, 4, 1, 8, true>;
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 1024, 0) ==
            hipSuccess &&
        per_cu > 0) {
    } else {
        cus = 256;
        per_cu = 1;
    }
    TrajArgs b = a;
    b.slots_per_lane = (uint32_t)kSlotsPerLane;
    hipLaunchKernelGGL(k, dim3(cus * per_cu), dim3(1024), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_trajectories(const TrajArgs& a, bool batched, const LaunchShape& shape, hipStream_t s) {
    const int vi = (shape.variant >= 0 && shape.variant < trajectory_variants()) ? shape.variant : 0;
    const Variant& v = kVariants[vi];
    TrajArgs b = a;
    b.slots_per_lane = v.spl;
    if (batched)
        v.launch_batch(dim3(shape.grid), dim3(v.block), s, b);
    else if (a.runout_angle)
        v.launch_single(dim3(shape.grid), dim3(v.block), s, b);
    else
        v.launch_single_plain(dim3(shape.grid), dim3(v.block), s, b);
    return hipGetLastError();
}

}  // namespace avl
