/*
 * CPU oracle for the avalanche overlay hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this code. The
 * product library never links, loads or calls it, and the two share no code: the GPU path is written
 * separately from the same model definition.
 *
 * Plain, slow, single-threaded C11. One source gives two twins:
 *   - the FP32 oracle (default): every operation is IEEE binary32, round to nearest, evaluated in the
 *     written order; build with -ffp-contract=off -fno-fast-math so no FMA is formed;
 *   - the FP64 twin (-DAVL_F64): the same text in binary64, used to state the FP32 error.
 * Inputs (the DEM, parameters) are float in both twins; the twin converts them exactly to double.
 *
 * What the paper fixes (section 5.2, Avalanches): a normals node over the DEM texels; a release-point
 * node that keeps texels whose steepness lies in a user range; a trajectory node that releases a
 * user-set number of particles per release texel and moves every particle with a persistence ratio
 * (momentum), a user-set amount of random deviation from the optimal path and a runout-angle stop;
 * its output is a per-texel velocity indicator (the maximal vertical displacement per step, figure 4)
 * and the spread of mass. The paper gives no equations; the definitions below are the readings
 * listed in the design notes (friction law, direction blend, random draw, accumulation, boundaries).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef AVL_F64
typedef double real;
#define SQRT sqrt
#define FLOOR floor
#define NAME(x) x##_f64
#else
typedef float real;
#define SQRT sqrtf
#define FLOOR floorf
#define NAME(x) x##_f32
#endif

#define R(v) ((real)(v))

/* ----------------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * Ten rounds of the 4x32 bijection; each round multiplies words 0 and 2 by the two Philox constants,
 * takes 64-bit products apart into high and low halves, and mixes in words 1 and 3 and the round key.
 * The key is bumped by the two Weyl constants between rounds.
 * ---------------------------------------------------------------------------------------------- */
void NAME(oracle_philox4x32_10)(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in [0, 1) with 24 random bits: exact in binary32 and binary64. */
static real unit24(uint32_t u) { return (real)(u >> 8) * R(0x1p-24); }

/* The two uniforms of step n of particle (cell, replica) in run `run`: one Philox block serves two
 * consecutive steps; even steps take words 0 and 1, odd steps words 2 and 3. Counter = (n/2, replica,
 * index of the release texel in the release texture (r*W+c at the DEM's resolution), run), key = the
 * 64-bit seed as (low, high) words. */
static void draw(uint32_t n, uint32_t replica, uint32_t cell, uint32_t run, uint64_t seed, real* rx, real* ry)
{
    uint32_t ctr[4] = {n >> 1, replica, cell, run};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    NAME(oracle_philox4x32_10)(ctr, key, o);
    uint32_t ux = (n & 1u) ? o[2] : o[0];
    uint32_t uy = (n & 1u) ? o[3] : o[1];
    *rx = R(2) * unit24(ux) - R(1);
    *ry = R(2) * unit24(uy) - R(1);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ----------------------------------------------------------------------------------------------
 * Normals and steepness (section 5.2: the normals node, per DEM texel; section 5.1 uses the same
 * node). Gradient by the textbook finite difference: central (z[i+1]-z[i-1])/(2 cs) inside, one-sided
 * (z[1]-z[0])/cs and (z[n-1]-z[n-2])/cs at the two edges. x runs along columns, y along rows.
 * Unit normal n = (-gx, -gy, 1)/sqrt(gx^2+gy^2+1). Channel 3 is the slope angle in degrees, for display.
 * Output: 4 reals per cell, row-major.
 * ---------------------------------------------------------------------------------------------- */
void NAME(oracle_normals)(const float* dem, int H, int W, float cell_size, real* out4)
{
    const real cs = (real)cell_size;
    const real cs2 = R(2) * cs;
    for (int r = 0; r < H; ++r) {
        for (int c = 0; c < W; ++c) {
            real gx, gy;
            if (c == 0)          gx = ((real)dem[(size_t)r * W + 1] - (real)dem[(size_t)r * W]) / cs;
            else if (c == W - 1) gx = ((real)dem[(size_t)r * W + W - 1] - (real)dem[(size_t)r * W + W - 2]) / cs;
            else                 gx = ((real)dem[(size_t)r * W + c + 1] - (real)dem[(size_t)r * W + c - 1]) / cs2;
            if (r == 0)          gy = ((real)dem[(size_t)W + c] - (real)dem[c]) / cs;
            else if (r == H - 1) gy = ((real)dem[(size_t)(H - 1) * W + c] - (real)dem[(size_t)(H - 2) * W + c]) / cs;
            else                 gy = ((real)dem[(size_t)(r + 1) * W + c] - (real)dem[(size_t)(r - 1) * W + c]) / cs2;
            real gg = gx * gx + gy * gy;
            real l = SQRT(gg + R(1));
            real* o = out4 + 4 * ((size_t)r * W + c);
            o[0] = -(gx / l);
            o[1] = -(gy / l);
            o[2] = R(1) / l;
            o[3] = (real)(atan(sqrt((double)gg)) * (180.0 / 3.14159265358979323846));
        }
    }
}

/* ----------------------------------------------------------------------------------------------
 * Release mask (section 5.2: the release-point node keeps texels whose steepness lies in the user's
 * range; the elevation window is an added criterion). Steepness theta lies in [smin, smax] exactly
 * when nz = cos(theta) lies in [cos(smax), cos(smin)]; the two cosines are taken in binary64 from
 * degrees * (pi/180) and rounded once to the working precision. Bounds are inclusive.
 * ---------------------------------------------------------------------------------------------- */
void NAME(oracle_release_mask)(const real* normals4, const float* dem, int H, int W, float smin_deg,
                               float smax_deg, float z_min, float z_max, uint8_t* mask)
{
    const double d2r = 3.14159265358979323846 / 180.0;
    const real cmin = (real)cos((double)smax_deg * d2r);
    const real cmax = (real)cos((double)smin_deg * d2r);
    for (size_t i = 0; i < (size_t)H * W; ++i) {
        real nz = normals4[4 * i + 2];
        real z = (real)dem[i];
        mask[i] = (cmin <= nz && nz <= cmax && (real)z_min <= z && z <= (real)z_max) ? 1 : 0;
    }
}

/* Release map at a finer texture resolution (section 5.2: the user picks the texture resolution at which
 * release points are evaluated). The release texture has mult x mult texels per DEM cell; texel (R, C) of
 * the (mult*H) x (mult*W) grid is centred at ((C + 1/2) / mult, (R + 1/2) / mult) in DEM cell units. There
 * nz and the elevation are read with bilinear filtering between texel centres and clamped indices (what a
 * texture sampler with linear filtering and clamp-to-edge addressing returns), and the test of
 * oracle_release_mask is applied to the filtered values. nz is filtered as a scalar, not renormalised. With
 * mult = 1 every centre falls on a texel centre, the weights are zero and the map is oracle_release_mask's. */
void NAME(oracle_release_mask_fine)(const real* normals4, const float* dem, int H, int W, int mult,
                                    float smin_deg, float smax_deg, float z_min, float z_max, uint8_t* mask)
{
    const double d2r = 3.14159265358979323846 / 180.0;
    const real cmin = (real)cos((double)smax_deg * d2r);
    const real cmax = (real)cos((double)smin_deg * d2r);
    const int Hf = H * mult, Wf = W * mult;
    for (int rr = 0; rr < Hf; ++rr)
        for (int cc = 0; cc < Wf; ++cc) {
            real x = ((real)cc + R(0.5)) / (real)mult, y = ((real)rr + R(0.5)) / (real)mult;
            real sx = x - R(0.5), sy = y - R(0.5);
            real fc = FLOOR(sx), fr = FLOOR(sy);
            real fx = sx - fc, fy = sy - fr;
            int c0 = (int)fc, r0 = (int)fr;
            size_t ca = (size_t)clampi(c0, 0, W - 1), cb = (size_t)clampi(c0 + 1, 0, W - 1);
            size_t ra = (size_t)clampi(r0, 0, H - 1), rb = (size_t)clampi(r0 + 1, 0, H - 1);
            real n00 = normals4[4 * (ra * W + ca) + 2], n01 = normals4[4 * (ra * W + cb) + 2];
            real n10 = normals4[4 * (rb * W + ca) + 2], n11 = normals4[4 * (rb * W + cb) + 2];
            real ntop = n00 + fx * (n01 - n00), nbot = n10 + fx * (n11 - n10);
            real nz = ntop + fy * (nbot - ntop);
            real z00 = (real)dem[ra * W + ca], z01 = (real)dem[ra * W + cb];
            real z10 = (real)dem[rb * W + ca], z11 = (real)dem[rb * W + cb];
            real ztop = z00 + fx * (z01 - z00), zbot = z10 + fx * (z11 - z10);
            real z = ztop + fy * (zbot - ztop);
            mask[(size_t)rr * Wf + cc] =
                (cmin <= nz && nz <= cmax && (real)z_min <= z && z <= (real)z_max) ? 1 : 0;
        }
}

/* ----------------------------------------------------------------------------------------------
 * Snow cover (section 5.1): a per-texel decision from the terrain alone, with user parameters for the
 * snow line, the maximal steepness and the blending of the transition zones; the overlay is white with
 * the blend factor as its alpha. Reading: two linear ramps multiplied,
 *   elevation: a_z = 0 at z <= snow_line, rising to 1 at z >= snow_line + alt_blend (a step at the
 *              snow line when alt_blend = 0);
 *   steepness: a_s = 1 where the slope is at most max_slope - slope_blend, falling to 0 at max_slope,
 *              linear in nz = cos(slope) between the two host-rounded cosines (a step at max_slope when
 *              slope_blend = 0);
 *   alpha = a_z * a_s, in binary32, ramps as t = (v - lo) / (hi - lo) clamped to [0, 1] (NaN -> 0).
 * ---------------------------------------------------------------------------------------------- */
static real ramp(real v, real lo, real hi)
{
    if (!(hi > lo)) return v >= lo ? R(1) : R(0);
    real t = (v - lo) / (hi - lo);
    return t > 0 ? (t < 1 ? t : R(1)) : R(0);
}

void NAME(oracle_snow_cover)(const real* normals4, const float* dem, int H, int W, float snow_line,
                             float alt_blend, float max_slope_deg, float slope_blend_deg, real* alpha)
{
    const double d2r = 3.14159265358979323846 / 180.0;
    const real c_lo = (real)cos((double)max_slope_deg * d2r);                       /* nz at max_slope */
    const real c_hi = (real)cos(((double)max_slope_deg - (double)slope_blend_deg) * d2r); /* full cover */
    const real z_lo = (real)snow_line;
    const real z_hi = (real)snow_line + (real)alt_blend;
    for (size_t i = 0; i < (size_t)H * W; ++i) {
        real a_z = ramp((real)dem[i], z_lo, z_hi);
        real a_s = ramp(normals4[4 * i + 2], c_lo, c_hi);
        alpha[i] = a_z * a_s;
    }
}

/* Release-cell list: linear indices r*W+c of the set cells of the mask in row-major order. */
int64_t NAME(oracle_compact)(const uint8_t* mask, int H, int W, int32_t* cells)
{
    int64_t n = 0;
    for (size_t i = 0; i < (size_t)H * W; ++i)
        if (mask[i]) cells[n++] = (int32_t)i;
    return n;
}

/* ----------------------------------------------------------------------------------------------
 * Trajectory model (section 5.2, the trajectory node).
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    float mu;          /* Coulomb friction coefficient (>= 0) */
    float xi;          /* Voellmy turbulence coefficient in m/s^2 (> 0, +inf = no drag) */
    float flow_height; /* m (> 0) */
    float persistence; /* weight of the previous direction, [0, 1] */
    float randomness;  /* amplitude of the random deviation, >= 0 */
    float step_cells;  /* horizontal step length in cells (> 0) */
    float tan_alpha;   /* runout-angle stop: tan of the angle; < 0 disables */
    uint32_t flags;    /* unused by the oracle */
} oracle_params;

typedef struct {
    const float* dem;
    int H, W;
    real cs, g2, per, Q, rnd, L, dl2, mdl, cd, tca;
    int use_alpha;
    uint32_t S, run;
    uint64_t seed;
} model;

static void model_init(model* m, const float* dem, int H, int W, float cell_size, const oracle_params* p,
                       uint32_t S, uint64_t seed, uint32_t run)
{
    m->dem = dem; m->H = H; m->W = W;
    m->cs = (real)cell_size;
    const real g = R(9.81);
    m->g2 = g + g;                                    /* 2g */
    m->per = (real)p->persistence;
    m->Q = R(1) - m->per;                             /* weight of the downslope direction */
    m->rnd = (real)p->randomness;
    m->L = (real)p->step_cells;
    const real dl = m->L * m->cs;                     /* horizontal step length, m */
    m->dl2 = dl * dl;
    m->mdl = (real)p->mu * dl;                        /* Coulomb loss height per step, m */
    m->cd = m->g2 / ((real)p->xi * (real)p->flow_height); /* 2g/(xi h), 1/m; 0 when xi = +inf */
    m->use_alpha = p->tan_alpha >= 0.0f;
    m->tca = (real)p->tan_alpha * m->cs;
    m->S = S; m->run = run; m->seed = seed;
}

/* Bilinear height patch through the four texel centres around (x, y) (texel (r,c) sits at (c+.5, r+.5)),
 * indices clamped to the grid. Returns the height and its exact gradient (metres per cell). */
static void sample(const model* m, real x, real y, real* zz, real* gx, real* gy)
{
    real sx = x - R(0.5), sy = y - R(0.5);
    real fc = FLOOR(sx), fr = FLOOR(sy);
    real fx = sx - fc, fy = sy - fr;
    int c0 = (int)fc, r0 = (int)fr;
    int ca = clampi(c0, 0, m->W - 1), cb = clampi(c0 + 1, 0, m->W - 1);
    int ra = clampi(r0, 0, m->H - 1), rb = clampi(r0 + 1, 0, m->H - 1);
    real a = (real)m->dem[(size_t)ra * m->W + ca], b = (real)m->dem[(size_t)ra * m->W + cb];
    real c = (real)m->dem[(size_t)rb * m->W + ca], d = (real)m->dem[(size_t)rb * m->W + cb];
    real top = a + fx * (b - a);
    real bot = c + fx * (d - c);
    *zz = top + fy * (bot - top);
    *gx = (b - a) + fy * ((d - c) - (b - a));
    *gy = bot - top;
}

enum { END_LIMIT = 0, END_EXIT = 1, END_STOP = 2, END_ANGLE = 3 };

/* How a particle ended: the last position (x, y) with its v^2; for an energy stop, also the rejected
 * step's target (x1, y1) and numerator num <= 0. */
typedef struct {
    int reason;
    real x, y, v2;
    real x1, y1, num;
} end_info;

static void splat(const model* m, int64_t* q, real* f, real x, real y, real val);

#define TRACE_COLS 8 /* x, y, z, gx, gy, dx, dy, v2 */

/* One particle, replica `replica` of release texel (tr, tc) of a release texture with mult x mult texels
 * per DEM cell: it starts at the texel's centre ((tc + 1/2) / mult, (tr + 1/2) / mult) in DEM cell units,
 * inside DEM cell (tr / mult, tc / mult), and its random stream is keyed by the texel's index
 * tr * (mult * W) + tc in the release texture (mult = 1: the centre and index of DEM cell (tr, tc)). Adds
 * its cell entries to counts and its per-cell maximum of v^2 to vmax2 (either may be NULL). With a trace
 * buffer of (S+1) rows, row 0 is the released state and row n+1 the state after step n. Returns the end
 * reason; *steps gets the number of steps entered (the terminating one included); *rows the trace rows. */
static int particle_at(const model* m, int tr, int tc, int mult, uint32_t replica, uint32_t* counts, real* vmax2,
                       uint64_t* steps, real* trace, int64_t* rows, end_info* ei, int64_t* vel_q, real* vel,
                       real mp)
{
    const int W = m->W, H = m->H;
    const uint32_t cell_id = (uint32_t)tr * (uint32_t)(W * mult) + (uint32_t)tc;
    real x = ((real)tc + R(0.5)) / (real)mult, y = ((real)tr + R(0.5)) / (real)mult;
    real z, gx, gy;
    sample(m, x, y, &z, &gx, &gy);
    const real x0 = x, y0 = y, zr = z;
    /* initial direction: straight downslope (zero on flat ground) */
    real dx = 0, dy = 0;
    {
        real gg = gx * gx + gy * gy;
        if (gg > 0) {
            real t = R(1) / SQRT(gg);
            dx = -(gx * t);
            dy = -(gy * t);
        }
    }
    real v2 = 0;
    int cr = tr / mult, cc = tc / mult;
    if (counts) counts[(size_t)cr * W + cc] += 1; /* entry into the release cell, with v = 0 */
    int64_t nrow = 0;
    if (trace) {
        real* t = trace + TRACE_COLS * nrow++;
        t[0] = x; t[1] = y; t[2] = z; t[3] = gx; t[4] = gy; t[5] = dx; t[6] = dy; t[7] = v2;
    }
    int reason = END_LIMIT;
    uint64_t n_steps = 0;
    for (uint32_t n = 0; n < m->S; ++n) {
        ++n_steps;
        /* direction: persistence * previous + (1 - persistence) * downslope + randomness * uniform square */
        real rx, ry;
        draw(n, replica, cell_id, m->run, m->seed, &rx, &ry);
        real gg = gx * gx + gy * gy;
        real t = gg > 0 ? m->Q / SQRT(gg) : R(0);
        real wx = (m->per * dx - t * gx) + m->rnd * rx;
        real wy = (m->per * dy - t * gy) + m->rnd * ry;
        real ww = wx * wx + wy * wy;
        if (ww > 0) {
            real s = R(1) / SQRT(ww);
            dx = wx * s;
            dy = wy * s;
        }
        /* move one step; leaving the grid ends the particle */
        real x1 = x + m->L * dx;
        real y1 = y + m->L * dy;
        real fc = FLOOR(x1), fr = FLOOR(y1);
        if (!(fc >= 0 && fc < (real)W && fr >= 0 && fr < (real)H)) { reason = END_EXIT; break; }
        real xs = x1, ys = y1; /* the rejected target, for an energy stop */
        real z1, gx1, gy1;
        sample(m, x1, y1, &z1, &gx1, &gy1);
        /* kinetic energy: gravity work minus Coulomb loss; Voellmy drag taken implicitly over the path */
        real dz = z - z1;
        real ds = SQRT(m->dl2 + dz * dz);
        real num = v2 + m->g2 * (dz - m->mdl);
        if (!(num > 0)) {
            reason = END_STOP;
            if (ei) { ei->x1 = xs; ei->y1 = ys; ei->num = num; }
            break;
        }
        real v2n = num / (R(1) + m->cd * ds);
        if (m->use_alpha) {
            real hx = x1 - x0, hy = y1 - y0;
            if ((zr - z1) < m->tca * SQRT(hx * hx + hy * hy)) { reason = END_ANGLE; break; }
        }
        x = x1; y = y1; z = z1; gx = gx1; gy = gy1; v2 = v2n;
        int ri = (int)fr, ci = (int)fc;
        if (ri != cr || ci != cc) {
            cr = ri; cc = ci;
            if (counts) counts[(size_t)cr * W + cc] += 1;
        }
        if (vmax2 && v2 > vmax2[(size_t)cr * W + cc]) vmax2[(size_t)cr * W + cc] = v2;
        if (vel_q || vel) splat(m, vel_q, vel, x, y, mp * SQRT(v2));
        if (trace) {
            real* tr = trace + TRACE_COLS * nrow++;
            tr[0] = x; tr[1] = y; tr[2] = z; tr[3] = gx; tr[4] = gy; tr[5] = dx; tr[6] = dy; tr[7] = v2;
        }
    }
    *steps += n_steps;
    if (rows) *rows = nrow;
    if (ei) {
        ei->reason = reason; ei->x = x; ei->y = y; ei->v2 = v2;
        /* only an energy stop has a rejected target (set above); the other ends rest where they are */
        if (reason != END_STOP) { ei->x1 = x; ei->y1 = y; ei->num = 0; }
    }
    return reason;
}

/* a particle released at the centre of DEM cell (r, c) */
static int particle(const model* m, int r, int c, uint32_t replica, uint32_t* counts, real* vmax2,
                    uint64_t* steps, real* trace, int64_t* rows, end_info* ei, int64_t* vel_q, real* vel, real mp)
{
    return particle_at(m, r, c, 1, replica, counts, vmax2, steps, trace, rows, ei, vel_q, vel, mp);
}

/* Whole run from a release texture with mult x mult texels per DEM cell (mask: (mult*H) x (mult*W)):
 * particles_per_cell replicas from every set texel, texels in row-major order. counts (u32) and vmax
 * (real) are H*W DEM rasters, fully overwritten; vmax is sqrt of the per-cell max of v^2 (0 where no
 * particle came). stats (may be NULL) gets {steps, ended by grid exit, by stop, by limit}. */
int NAME(oracle_trajectories_fine)(const float* dem, const uint8_t* mask, int H, int W, int mult,
                                   float cell_size, const oracle_params* p, uint32_t particles_per_cell,
                                   uint32_t step_limit, uint64_t seed, uint32_t run, uint32_t* counts, real* vmax,
                                   uint64_t* stats)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    const size_t N = (size_t)H * W;
    const int Hf = H * mult, Wf = W * mult;
    memset(counts, 0, N * sizeof(uint32_t));
    for (size_t i = 0; i < N; ++i) vmax[i] = 0; /* holds v^2 until the end */
    uint64_t st[4] = {0, 0, 0, 0};
    for (int r = 0; r < Hf; ++r)
        for (int c = 0; c < Wf; ++c) {
            if (!mask[(size_t)r * Wf + c]) continue;
            for (uint32_t j = 0; j < particles_per_cell; ++j) {
                int why = particle_at(&m, r, c, mult, j, counts, vmax, &st[0], NULL, NULL, NULL, NULL, NULL, 0);
                st[why == END_EXIT ? 1 : (why == END_LIMIT ? 3 : 2)] += 1;
            }
        }
    for (size_t i = 0; i < N; ++i) vmax[i] = SQRT(vmax[i]);
    if (stats) memcpy(stats, st, sizeof st);
    return 0;
}

/* Whole run from a release map at the DEM's resolution: particles_per_cell replicas from the centre of
 * every set cell of the mask (H*W), cells in row-major order. */
int NAME(oracle_trajectories)(const float* dem, const uint8_t* mask, int H, int W, float cell_size,
                              const oracle_params* p, uint32_t particles_per_cell, uint32_t step_limit,
                              uint64_t seed, uint32_t run, uint32_t* counts, real* vmax, uint64_t* stats)
{
    return NAME(oracle_trajectories_fine)(dem, mask, H, W, 1, cell_size, p, particles_per_cell, step_limit, seed,
                                          run, counts, vmax, stats);
}

/* Trace of one particle (replica `replica` of release texel (tr, tc) at mult texels per DEM cell, as in
 * particle_at): trace must hold (step_limit+1)*8 reals. Returns the number of rows written;
 * *reason gets 0 (step limit), 1 (left the grid) or 2 (stopped); *steps the steps entered. */
int64_t NAME(oracle_trace_fine)(const float* dem, int H, int W, float cell_size, const oracle_params* p,
                                int tr, int tc, int mult, uint32_t replica, uint32_t step_limit, uint64_t seed,
                                uint32_t run, real* trace, int32_t* reason, uint64_t* steps)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    int64_t rows = 0;
    uint64_t st = 0;
    *reason = particle_at(&m, tr, tc, mult, replica, NULL, NULL, &st, trace, &rows, NULL, NULL, NULL, 0);
    if (*reason == END_ANGLE) *reason = END_STOP;
    *steps = st;
    return rows;
}

/* the same for a particle released at the centre of DEM cell (r, c) */
int64_t NAME(oracle_trace)(const float* dem, int H, int W, float cell_size, const oracle_params* p,
                           int r, int c, uint32_t replica, uint32_t step_limit, uint64_t seed, uint32_t run,
                           real* trace, int32_t* reason, uint64_t* steps)
{
    return NAME(oracle_trace_fine)(dem, H, W, cell_size, p, r, c, 1, replica, step_limit, seed, run, trace, reason,
                                   steps);
}

/* ----------------------------------------------------------------------------------------------
 * Smooth variant: deposit of the released mass where each particle comes to rest, and its gradient.
 *
 * Every particle of release cell c carries mp = mass[c] / P. It rests at p*:
 *   - energy stop during step n: the numerator of the energy step falls linearly from v^2 > 0 at the
 *     start of the step to num <= 0 at its end; its zero is at the fraction t* = v^2 / (v^2 - num) of
 *     the step (t* = 0 when v^2 = 0), so p* = p + t* (p1 - p);
 *   - runout-angle stop or step limit: p* = p;  leaving the grid: the mass is lost.
 * The deposit is the bilinear splat of mp at p* (the same four texel centres and weights as the height
 * sample; clamped corners merge), accumulated in fixed point q = rint(value * 2^24) as int64 so the raster
 * does not depend on the order of accumulation; `dep` (nullable) gets the same sum unquantised. With
 * vel_splat, every accepted step also splats mp * v at the particle's new position into vel_q / vel.
 * ---------------------------------------------------------------------------------------------- */
#ifdef AVL_F64
#define RINT_Q(v) llrint((v) * 0x1p24)
#else
#define RINT_Q(v) llrintf((v) * 0x1p24f)
#endif

typedef struct {
    int ca, cb, ra, rb;
    real fx, fy;
} corners;

static corners corners_of(const model* m, real x, real y)
{
    corners k;
    real sx = x - R(0.5), sy = y - R(0.5);
    real fc = FLOOR(sx), fr = FLOOR(sy);
    k.fx = sx - fc;
    k.fy = sy - fr;
    int c0 = (int)fc, r0 = (int)fr;
    k.ca = clampi(c0, 0, m->W - 1);
    k.cb = clampi(c0 + 1, 0, m->W - 1);
    k.ra = clampi(r0, 0, m->H - 1);
    k.rb = clampi(r0 + 1, 0, m->H - 1);
    return k;
}

static void splat(const model* m, int64_t* q, real* f, real x, real y, real val)
{
    corners k = corners_of(m, x, y);
    const real w[4] = {(R(1) - k.fx) * (R(1) - k.fy), k.fx * (R(1) - k.fy), (R(1) - k.fx) * k.fy, k.fx * k.fy};
    const size_t idx[4] = {(size_t)k.ra * m->W + k.ca, (size_t)k.ra * m->W + k.cb, (size_t)k.rb * m->W + k.ca,
                           (size_t)k.rb * m->W + k.cb};
    for (int i = 0; i < 4; ++i) {
        real v = val * w[i];
        if (q) q[idx[i]] += (int64_t)RINT_Q(v);
        if (f) f[idx[i]] += v;
    }
}

/* resting point of a particle that ended with *e (energy stop: fractional step) */
static void rest_point(const end_info* e, real* px, real* py, real* tstar)
{
    real t = 0;
    *px = e->x;
    *py = e->y;
    if (e->reason == END_STOP) {
        if (e->v2 > 0) t = e->v2 / (e->v2 - e->num);
        *px = e->x + t * (e->x1 - e->x);
        *py = e->y + t * (e->y1 - e->y);
    }
    *tstar = t;
}

static real mass_of(const float* mass, size_t cell) { return mass ? (real)mass[cell] : R(1); }

int NAME(oracle_smooth_forward)(const float* dem, const uint8_t* mask, const float* mass, int H, int W,
                                float cell_size, const oracle_params* p, uint32_t P, uint32_t step_limit,
                                uint64_t seed, uint32_t run, int vel_splat, int64_t* dep_q, real* dep,
                                int64_t* vel_q, real* vel, uint64_t* stats)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    const size_t N = (size_t)H * W;
    memset(dep_q, 0, N * sizeof(int64_t));
    if (dep) for (size_t i = 0; i < N; ++i) dep[i] = 0;
    if (vel_q) memset(vel_q, 0, N * sizeof(int64_t));
    if (vel) for (size_t i = 0; i < N; ++i) vel[i] = 0;
    uint64_t st[4] = {0, 0, 0, 0};
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            const size_t cell = (size_t)r * W + c;
            if (!mask[cell]) continue;
            const real mp = mass_of(mass, cell) / (real)P;
            for (uint32_t j = 0; j < P; ++j) {
                end_info e;
                int why = particle(&m, r, c, j, NULL, NULL, &st[0], NULL, NULL, &e, vel_splat ? vel_q : NULL,
                                   vel_splat ? vel : NULL, mp);
                st[why == END_EXIT ? 1 : (why == END_LIMIT ? 3 : 2)] += 1;
                if (why == END_EXIT) continue;
                real px, py, t;
                rest_point(&e, &px, &py, &t);
                splat(&m, dep_q, dep, px, py, mp);
            }
        }
    if (stats) memcpy(stats, st, sizeof st);
    return 0;
}

/* ----------------------------------------------------------------------------------------------
 * Gradient of a loss L(D) of the deposit, given gD = dL/dD per texel, with respect to mu, xi, h and
 * the release mass of every cell.
 *
 * Paths do not depend on mu, xi, h or the mass (the direction never reads the speed), so for each
 * particle only v^2 along its path and the fractional last step depend on (mu, xi, h):
 *   dL/dp*  = mp * sum over the splat corners of gD * grad w;  dL/dt* = dL/dp* . (p1 - p);
 *   t* = v2 / Dn with Dn = v2 - num = -2g (dz - mu dl), so dL/dv2_n = dL/dt* / Dn and the direct
 *   term dL/dmu += -dL/dt* * v2 * (2g dl) / Dn^2;
 *   reverse sweep of v2_{k+1} = (v2_k + 2g (dz_k - mu dl)) / (1 + a_k), a_k = 2g ds_k / (xi h):
 *     dL/dmu += lam_{k+1} * (-(2g dl) / (1 + a_k)); dL/dxi += lam_{k+1} * v2_{k+1} a_k / (xi (1 + a_k));
 *     dL/dh += lam_{k+1} * v2_{k+1} a_k / (h (1 + a_k)); lam_k = lam_{k+1} / (1 + a_k).
 * The mass enters linearly: dL/dmass[c] = (1/P) sum over c's particles of sum gD * w(p*).
 * A particle that stopped on the runout angle or the step limit rests at a point that does not move
 * with (mu, xi, h); one that left the grid deposits nothing.
 * Per-particle values (nullable, 4 reals per particle in release order: dmu, dxi, dh, sum gD w) are
 * in the working precision; the totals are summed in binary64 in particle order.
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    real gpx, gpy, gw; /* dL/dp* per unit mass (x, y) and sum gD * w at p* */
} splat_grad;

static splat_grad splat_gradient(const model* m, const float* gD, real px, real py)
{
    corners k = corners_of(m, px, py);
    const real g00 = (real)gD[(size_t)k.ra * m->W + k.ca], g01 = (real)gD[(size_t)k.ra * m->W + k.cb];
    const real g10 = (real)gD[(size_t)k.rb * m->W + k.ca], g11 = (real)gD[(size_t)k.rb * m->W + k.cb];
    splat_grad s;
    s.gpx = ((g01 - g00) * (R(1) - k.fy)) + ((g11 - g10) * k.fy);
    s.gpy = ((g10 - g00) * (R(1) - k.fx)) + ((g11 - g01) * k.fx);
    const real w00 = (R(1) - k.fx) * (R(1) - k.fy), w01 = k.fx * (R(1) - k.fy);
    const real w10 = (R(1) - k.fx) * k.fy, w11 = k.fx * k.fy;
    s.gw = ((g00 * w00) + (g01 * w01)) + ((g10 * w10) + (g11 * w11));
    return s;
}

int NAME(oracle_smooth_backward)(const float* dem, const uint8_t* mask, const float* mass, int H, int W,
                                 float cell_size, const oracle_params* p, uint32_t P, uint32_t step_limit,
                                 uint64_t seed, uint32_t run, const float* gD, double* gparams, double* gmass,
                                 real* per_particle)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    const size_t N = (size_t)H * W;
    real* trace = (real*)malloc(sizeof(real) * TRACE_COLS * ((size_t)step_limit + 1));
    if (!trace) return -1;
    const real g2dl = m.g2 * (m.L * m.cs);
    const real xi = (real)p->xi, h = (real)p->flow_height;
    double gmu = 0, gxi = 0, gh = 0;
    for (size_t i = 0; i < N; ++i) gmass[i] = 0;
    size_t k_out = 0;
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            const size_t cell = (size_t)r * W + c;
            if (!mask[cell]) continue;
            const real mp = mass_of(mass, cell) / (real)P;
            double gm_sum = 0;
            for (uint32_t j = 0; j < P; ++j) {
                end_info e;
                uint64_t st = 0;
                int64_t rows = 0;
                int why = particle(&m, r, c, j, NULL, NULL, &st, trace, &rows, &e, NULL, NULL, 0);
                real dmu = 0, dxi = 0, dh = 0, gw = 0;
                if (why != END_EXIT) {
                    real px, py, t;
                    rest_point(&e, &px, &py, &t);
                    splat_grad sg = splat_gradient(&m, gD, px, py);
                    gw = sg.gw;
                    if (why == END_STOP) {
                        const real gt = mp * ((sg.gpx * (e.x1 - e.x)) + (sg.gpy * (e.y1 - e.y)));
                        const real Dn = e.v2 - e.num;
                        real lam = 0;
                        if (Dn > 0) {
                            lam = gt / Dn;
                            dmu = -((gt * (e.v2 / Dn)) * (g2dl / Dn));
                        }
                        /* reverse sweep over the accepted steps k = rows-2 .. 0 */
                        for (int64_t k = rows - 2; k >= 0; --k) {
                            const real* a0 = trace + TRACE_COLS * k;
                            const real* a1 = trace + TRACE_COLS * (k + 1);
                            const real dz = a0[2] - a1[2];
                            const real ds = SQRT(m.dl2 + dz * dz);
                            const real a = m.cd * ds;
                            const real op = R(1) + a;
                            const real v2n = a1[7];
                            dmu = dmu - lam * (g2dl / op);
                            dxi = dxi + lam * ((v2n * a) / (xi * op));
                            dh = dh + lam * ((v2n * a) / (h * op));
                            lam = lam / op;
                        }
                    }
                }
                gmu += (double)dmu;
                gxi += (double)dxi;
                gh += (double)dh;
                gm_sum += (double)gw;
                if (per_particle) {
                    real* o = per_particle + 4 * k_out;
                    o[0] = dmu; o[1] = dxi; o[2] = dh; o[3] = gw;
                }
                ++k_out;
            }
            gmass[cell] = gm_sum / (double)P;
        }
    free(trace);
    gparams[0] = gmu;
    gparams[1] = gxi;
    gparams[2] = gh;
    return 0;
}

/* Forward-mode derivation of the same (mu, xi, h) gradient, independent of the reverse sweep: the
 * tangents dv2/dmu, dv2/dxi, dv2/dh are carried forward along each path,
 *   dv2_{k+1}/dmu = (dv2_k/dmu - 2g dl) / (1 + a_k),
 *   dv2_{k+1}/dxi = dv2_k/dxi / (1 + a_k) + v2_{k+1} a_k / (xi (1 + a_k))  (h likewise),
 * and at an energy stop d(t*)/d(theta) = (dv2_n/d(theta)) / Dn (+ the direct -v2 (2g dl) / Dn^2 for mu);
 * dL/d(theta) = sum over particles of dL/d(t*) times d(t*)/d(theta). Binary64 only. */
#ifdef AVL_F64
int oracle_smooth_tangent_f64(const float* dem, const uint8_t* mask, const float* mass, int H, int W,
                              float cell_size, const oracle_params* p, uint32_t P, uint32_t step_limit,
                              uint64_t seed, uint32_t run, const float* gD, double* gparams)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    real* trace = (real*)malloc(sizeof(real) * TRACE_COLS * ((size_t)step_limit + 1));
    if (!trace) return -1;
    const real g2dl = m.g2 * (m.L * m.cs);
    const real xi = (real)p->xi, h = (real)p->flow_height;
    double out[3] = {0, 0, 0};
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            const size_t cell = (size_t)r * W + c;
            if (!mask[cell]) continue;
            const real mp = mass_of(mass, cell) / (real)P;
            for (uint32_t j = 0; j < P; ++j) {
                end_info e;
                uint64_t st = 0;
                int64_t rows = 0;
                int why = particle(&m, r, c, j, NULL, NULL, &st, trace, &rows, &e, NULL, NULL, 0);
                if (why != END_STOP) continue;
                double tmu = 0, txi = 0, th = 0; /* tangents of v2 */
                for (int64_t k = 0; k + 1 < rows; ++k) {
                    const real* a0 = trace + TRACE_COLS * k;
                    const real* a1 = trace + TRACE_COLS * (k + 1);
                    const double dz = a0[2] - a1[2];
                    const double ds = sqrt(m.dl2 + dz * dz);
                    const double a = m.cd * ds;
                    const double v2n = a1[7];
                    tmu = (tmu - g2dl) / (1 + a);
                    txi = txi / (1 + a) + v2n * a / (xi * (1 + a));
                    th = th / (1 + a) + v2n * a / (h * (1 + a));
                }
                const double Dn = e.v2 - e.num;
                if (!(Dn > 0)) continue;
                real px, py, t;
                rest_point(&e, &px, &py, &t);
                splat_grad sg = splat_gradient(&m, gD, px, py);
                const double gt = mp * (sg.gpx * (e.x1 - e.x) + sg.gpy * (e.y1 - e.y));
                out[0] += gt * (tmu / Dn - e.v2 * g2dl / (Dn * Dn));
                out[1] += gt * (txi / Dn);
                out[2] += gt * (th / Dn);
            }
        }
    free(trace);
    gparams[0] = out[0];
    gparams[1] = out[1];
    gparams[2] = out[2];
    return 0;
}
#endif

/* Per-particle view of the smooth deposit, for finite-difference checks of the gradient: for every
 * particle (release order), its share of L = sum gD * D (mp * sum over the splat corners of gD * w at the
 * resting point), its end reason and the number of steps it completed. */
int NAME(oracle_smooth_particles)(const float* dem, const uint8_t* mask, const float* mass, int H, int W,
                                  float cell_size, const oracle_params* p, uint32_t P, uint32_t step_limit,
                                  uint64_t seed, uint32_t run, const float* gD, double* Lp, int32_t* reason,
                                  int32_t* steps_done)
{
    model m;
    model_init(&m, dem, H, W, cell_size, p, step_limit, seed, run);
    real* trace = (real*)malloc(sizeof(real) * TRACE_COLS * ((size_t)step_limit + 1));
    if (!trace) return -1;
    size_t k = 0;
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            const size_t cell = (size_t)r * W + c;
            if (!mask[cell]) continue;
            const real mp = mass_of(mass, cell) / (real)P;
            for (uint32_t j = 0; j < P; ++j, ++k) {
                end_info e;
                uint64_t st = 0;
                int64_t rows = 0;
                int why = particle(&m, r, c, j, NULL, NULL, &st, trace, &rows, &e, NULL, NULL, 0);
                reason[k] = why;
                steps_done[k] = (int32_t)(rows - 1);
                Lp[k] = 0;
                if (why == END_EXIT) continue;
                real px, py, t;
                rest_point(&e, &px, &py, &t);
                splat_grad sg = splat_gradient(&m, gD, px, py);
                Lp[k] = (double)mp * (double)sg.gw;
            }
        }
    free(trace);
    return 0;
}

/* ----------------------------------------------------------------------------------------------
 * Multi-resolution overlay (section 3: a mipmap is computed from the full-resolution overlay).
 * Level l + 1 halves level l, rounding up: cell (r, c) of level l + 1 covers cells 2r..2r+1 x
 * 2c..2c+1 of level l, those that exist. Entry counts add (64-bit); speeds take the maximum.
 * Levels 1 .. n_levels - 1 are written one after the other, each row-major.
 * ---------------------------------------------------------------------------------------------- */
int64_t NAME(oracle_mipmap)(const uint32_t* counts, const float* vmax, int H, int W, int n_levels, uint64_t* cpyr,
                            float* vpyr)
{
    int h = H, w = W;
    int64_t at = 0, prev = -1; /* start of the previous level in the output (-1: the input) */
    for (int l = 1; l < n_levels; ++l) {
        const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
        for (int r = 0; r < h2; ++r)
            for (int c = 0; c < w2; ++c) {
                uint64_t sum = 0;
                float mx = 0.0f;
                for (int dr = 0; dr < 2; ++dr)
                    for (int dc = 0; dc < 2; ++dc) {
                        const int rr = 2 * r + dr, cc = 2 * c + dc;
                        if (rr >= h || cc >= w) continue;
                        const size_t i = (size_t)rr * w + cc;
                        const uint64_t cnt = prev < 0 ? (uint64_t)counts[i] : cpyr[prev + i];
                        const float v = prev < 0 ? vmax[i] : vpyr[prev + i];
                        sum += cnt;
                        if (v > mx) mx = v;
                    }
                cpyr[at + (size_t)r * w2 + c] = sum;
                vpyr[at + (size_t)r * w2 + c] = mx;
            }
        prev = at;
        at += (int64_t)h2 * w2;
        h = h2;
        w = w2;
    }
    return at;
}
