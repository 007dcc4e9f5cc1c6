// Terrain passes of the avalanche overlay (section 5.2 of arXiv 2506.23364): surface normals and
// steepness per DEM texel, the release-point map from a steepness range and an elevation window, and
// the row-major list of release texels. Plus the fill, padded-DEM and finalize helpers of the trajectory
// pass.
//
// These are streaming passes, written for 64-wide wavefronts with every wave touching whole 256-byte
// stretches of consecutive cells; all but the normals (bound by their correctly rounded arithmetic) are
// bound by HBM bandwidth.
#include "avl_internal.h"

namespace avl {

// ------------------------------------------------------------------------------------------ normals
// Block = 64 x 16 texels, 256 threads (one wave per row, four rows per thread); the tile plus a
// one-texel halo is staged in LDS so every DEM value is read from L2/HBM about once. Gradient: central
// difference inside, one-sided at the grid edges (the textbook finite difference);
// n = (-gx, -gy, 1)/sqrt(gx^2 + gy^2 + 1). Each texel takes five correctly rounded divisions, two square
// roots and an arctangent, so the pass is bound by VALU issue; a thread's four texels are independent
// chains the compiler interleaves.
// kMask: the release map of the same texels as well (the release-mask pass below on the nz just computed and
// the staged height, so the map is the one that pass writes from these normals, without reading them back).
struct MaskArgs {
    float cmin, cmax, zmin, zmax;
    uint8_t* mask;
};
constexpr int kNTX = 64, kNTY = 16, kNRows = 4;  // tile columns, tile rows, rows of threads
template <bool kMask>
__global__ __launch_bounds__(kNTX * kNRows) void k_normals(const float* __restrict__ dem, int H, int W, float cs,
                                                           float cs2, float4* __restrict__ out, MaskArgs m) {
    __shared__ float tile[kNTY + 2][kNTX + 2];
    const int tx = threadIdx.x & (kNTX - 1), ty = threadIdx.x / kNTX;
    const int c0 = blockIdx.x * kNTX, r0 = blockIdx.y * kNTY;
    // stage (kNTY + 2) x (kNTX + 2) texels with clamped indices
    for (int i = threadIdx.x; i < (kNTY + 2) * (kNTX + 2); i += kNTX * kNRows) {
        int lr = i / (kNTX + 2), lc = i - lr * (kNTX + 2);
        int r = min(max(r0 + lr - 1, 0), H - 1);
        int c = min(max(c0 + lc - 1, 0), W - 1);
        tile[lr][lc] = dem[(size_t)r * W + c];
    }
    __syncthreads();
    const int c = c0 + tx;
    if (c >= W) return;
#pragma unroll
    for (int k = 0; k < kNTY / kNRows; ++k) {
        const int r = r0 + ty + k * kNRows;
        if (r >= H) break;
        const int lr = ty + k * kNRows + 1, lc = tx + 1;
        float gx, gy;
        if (c == 0)
            gx = (tile[lr][lc + 1] - tile[lr][lc]) / cs;
        else if (c == W - 1)
            gx = (tile[lr][lc] - tile[lr][lc - 1]) / cs;
        else
            gx = (tile[lr][lc + 1] - tile[lr][lc - 1]) / cs2;
        if (r == 0)
            gy = (tile[lr + 1][lc] - tile[lr][lc]) / cs;
        else if (r == H - 1)
            gy = (tile[lr][lc] - tile[lr - 1][lc]) / cs;
        else
            gy = (tile[lr + 1][lc] - tile[lr - 1][lc]) / cs2;
        const float gg = gx * gx + gy * gy;
        const float l = sqrtf(gg + 1.0f);
        float4 o;
        o.x = -(gx / l);
        o.y = -(gy / l);
        o.z = 1.0f / l;
        o.w = atanf(sqrtf(gg)) * 57.295779513082320876798f;
        out[(size_t)r * W + c] = o;
        if constexpr (kMask) {
            const float z = tile[lr][lc];  // dem[r][c]: an in-grid texel is staged unclamped
            m.mask[(size_t)r * W + c] = (m.cmin <= o.z && o.z <= m.cmax && m.zmin <= z && z <= m.zmax) ? 1 : 0;
        }
    }
}

hipError_t launch_normals(const float* dem, int H, int W, float cs, float* out4, hipStream_t s) {
    dim3 grid((W + kNTX - 1) / kNTX, (H + kNTY - 1) / kNTY);
    const float cs2 = 2.0f * cs;
    hipLaunchKernelGGL(k_normals<false>, grid, dim3(kNTX * kNRows), 0, s, dem, H, W, cs, cs2,
                       reinterpret_cast<float4*>(out4), MaskArgs{});
    return hipGetLastError();
}

hipError_t launch_normals_mask(const float* dem, int H, int W, float cs, float cmin, float cmax, float zmin,
                               float zmax, float* out4, uint8_t* mask, hipStream_t s) {
    dim3 grid((W + kNTX - 1) / kNTX, (H + kNTY - 1) / kNTY);
    const float cs2 = 2.0f * cs;
    hipLaunchKernelGGL(k_normals<true>, grid, dim3(kNTX * kNRows), 0, s, dem, H, W, cs, cs2,
                       reinterpret_cast<float4*>(out4), MaskArgs{cmin, cmax, zmin, zmax, mask});
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ release mask
// Four texels per thread: one 16-byte load of each normal, one 16-byte load of four heights when the
// four are in range, one 4-byte store of four mask bytes.
__global__ __launch_bounds__(256) void k_release_mask(const float4* __restrict__ nrm, const float* __restrict__ dem,
                                                      int64_t n, float cmin, float cmax, float zmin, float zmax,
                                                      uint8_t* __restrict__ mask) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    if (i0 + 4 <= n) {
        uint32_t packed = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float nz = nrm[i0 + k].z;
            const float z = dem[i0 + k];
            const uint32_t m = (cmin <= nz && nz <= cmax && zmin <= z && z <= zmax) ? 1u : 0u;
            packed |= m << (8 * k);
        }
        if ((reinterpret_cast<uintptr_t>(mask + i0) & 3) == 0) {
            *reinterpret_cast<uint32_t*>(mask + i0) = packed;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) mask[i0 + k] = (uint8_t)(packed >> (8 * k));
        }
    } else {
        for (int64_t i = i0; i < n; ++i) {
            const float nz = nrm[i].z;
            const float z = dem[i];
            mask[i] = (cmin <= nz && nz <= cmax && zmin <= z && z <= zmax) ? 1 : 0;
        }
    }
}

hipError_t launch_release_mask(const float* normals4, const float* dem, int64_t n, float cmin, float cmax,
                               float zmin, float zmax, uint8_t* mask, hipStream_t s) {
    const int64_t threads = (n + 3) / 4;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_release_mask, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(normals4), dem, n, cmin, cmax, zmin, zmax, mask);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ snow cover
// alpha = ramp(z; snow line, + alt blend) * ramp(nz; cos max slope, cos(max slope - slope blend)), a ramp
// being (v - lo) / (hi - lo) clamped to [0, 1] (NaN -> 0), or the step v >= lo when hi <= lo. Four texels
// per thread: four 16-byte normal loads, one 16-byte height load, one 16-byte alpha store.
__device__ __forceinline__ float snow_ramp(float v, float lo, float hi, bool step) {
    if (step) return v >= lo ? 1.0f : 0.0f;
    const float t = (v - lo) / (hi - lo);
    return t > 0.0f ? (t < 1.0f ? t : 1.0f) : 0.0f;
}

__global__ __launch_bounds__(256) void k_snow_cover(const float4* __restrict__ nrm, const float* __restrict__ dem,
                                                    int64_t n, float z_lo, float z_hi, float c_lo, float c_hi,
                                                    float* __restrict__ alpha) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    const bool zstep = !(z_hi > z_lo), cstep = !(c_hi > c_lo);
    if (i0 + 4 <= n && (reinterpret_cast<uintptr_t>(dem + i0) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(alpha + i0) & 15) == 0) {
        const float4 z4 = *reinterpret_cast<const float4*>(dem + i0);
        const float z[4] = {z4.x, z4.y, z4.z, z4.w};
        float a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a[k] = snow_ramp(z[k], z_lo, z_hi, zstep) * snow_ramp(nrm[i0 + k].z, c_lo, c_hi, cstep);
        *reinterpret_cast<float4*>(alpha + i0) = make_float4(a[0], a[1], a[2], a[3]);
    } else {
        for (int64_t i = i0; i < n && i < i0 + 4; ++i)
            alpha[i] = snow_ramp(dem[i], z_lo, z_hi, zstep) * snow_ramp(nrm[i].z, c_lo, c_hi, cstep);
    }
}

hipError_t launch_snow_cover(const float* normals4, const float* dem, int64_t n, float z_lo, float z_hi, float c_lo,
                             float c_hi, float* alpha, hipStream_t s) {
    const int64_t threads = (n + 3) / 4;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_snow_cover, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const float4*>(normals4), dem, n,
                       z_lo, z_hi, c_lo, c_hi, alpha);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ fine release map
// Release texture with mult x mult texels per DEM cell: texel (R, C) is centred at ((C + 1/2) / mult,
// (R + 1/2) / mult) in DEM cell units, where nz and the height are filtered bilinearly between texel centres
// with clamped indices and tested against the same bounds as the plain map. A block covers kFineSpan
// consecutive texels of one row (row and span from the block index, once per block). The block first
// stages nz and the height of the two DEM rows and the column range its texels touch in LDS (coalesced
// reads; the column range is exact because the texel centres and their floors grow with C), then each
// thread filters four texels from LDS and stores their four bytes at once.
constexpr int kFineThreads = 256;
constexpr int kFineSpan = 4 * kFineThreads;
constexpr int kFineCols = kFineSpan + 3;  // columns a span can touch at mult = 1 (kFineSpan + 1), with margin

__device__ __forceinline__ int fine_col(int64_t C, float fm) {  // floor(x - 1/2) of texel column C's centre
    const float x = ((float)C + 0.5f) / fm;
    return (int)floorf(x - 0.5f);
}

__global__ __launch_bounds__(kFineThreads) void k_release_mask_fine(const float4* __restrict__ nrm,
                                                                    const float* __restrict__ dem, int H, int W,
                                                                    int mult, uint32_t spans_per_row, float cmin,
                                                                    float cmax, float zmin, float zmax,
                                                                    uint8_t* __restrict__ mask) {
    __shared__ float s_n[2][kFineCols], s_z[2][kFineCols];
    const uint32_t rr = blockIdx.x / spans_per_row;  // uniform
    const uint32_t span = blockIdx.x - rr * spans_per_row;
    const int64_t Wf = (int64_t)W * mult;
    const int64_t cs0 = (int64_t)span * kFineSpan;
    const int64_t cs1 = min(cs0 + kFineSpan, Wf) - 1;  // last texel column of the span
    const float fm = (float)mult;
    const int lo = min(max(fine_col(cs0, fm), 0), W - 1);
    const int hi = min(max(fine_col(cs1, fm) + 1, 0), W - 1);
    const float y = ((float)rr + 0.5f) / fm;
    const float sy = y - 0.5f;
    const float fr = floorf(sy);
    const float fy = sy - fr;
    const int r0 = (int)fr;
    const int64_t ra = (int64_t)min(max(r0, 0), H - 1) * W;
    const int64_t rb = (int64_t)min(max(r0 + 1, 0), H - 1) * W;
    for (int k = threadIdx.x; k <= hi - lo; k += kFineThreads) {
        s_n[0][k] = nrm[ra + lo + k].z;
        s_n[1][k] = nrm[rb + lo + k].z;
        s_z[0][k] = dem[ra + lo + k];
        s_z[1][k] = dem[rb + lo + k];
    }
    __syncthreads();
    const int64_t c0 = cs0 + 4 * threadIdx.x;
    if (c0 >= Wf) return;
    uint32_t packed = 0;
    const int nk = (int)min((int64_t)4, Wf - c0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < nk) {
            const float x = ((float)(c0 + k) + 0.5f) / fm;
            const float sx = x - 0.5f;
            const float fc = floorf(sx);
            const float fx = sx - fc;
            const int cc = (int)fc;
            const int ca = min(max(cc, 0), W - 1) - lo, cb = min(max(cc + 1, 0), W - 1) - lo;
            const float n00 = s_n[0][ca], n01 = s_n[0][cb], n10 = s_n[1][ca], n11 = s_n[1][cb];
            const float ntop = n00 + fx * (n01 - n00), nbot = n10 + fx * (n11 - n10);
            const float nz = ntop + fy * (nbot - ntop);
            const float z00 = s_z[0][ca], z01 = s_z[0][cb], z10 = s_z[1][ca], z11 = s_z[1][cb];
            const float ztop = z00 + fx * (z01 - z00), zbot = z10 + fx * (z11 - z10);
            const float z = ztop + fy * (zbot - ztop);
            const uint32_t m = (cmin <= nz && nz <= cmax && zmin <= z && z <= zmax) ? 1u : 0u;
            packed |= m << (8 * k);
        }
    }
    uint8_t* out = mask + (int64_t)rr * Wf + c0;
    if (nk == 4 && (reinterpret_cast<uintptr_t>(out) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(out) = packed;
    } else {
        for (int k = 0; k < nk; ++k) out[k] = (uint8_t)(packed >> (8 * k));
    }
}

hipError_t launch_release_mask_fine(const float* normals4, const float* dem, int H, int W, int mult, float cmin,
                                    float cmax, float zmin, float zmax, uint8_t* mask, hipStream_t s) {
    const int64_t Wf = (int64_t)W * mult, Hf = (int64_t)H * mult;
    const int64_t spans = (Wf + kFineSpan - 1) / kFineSpan;
    const int64_t blocks = spans * Hf;  // < 2^31 / 1024 * 2 + Hf: fits a 32-bit grid
    hipLaunchKernelGGL(k_release_mask_fine, dim3((unsigned)blocks), dim3(kFineThreads), 0, s,
                       reinterpret_cast<const float4*>(normals4), dem, H, W, mult, (uint32_t)spans, cmin, cmax, zmin,
                       zmax, mask);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ compaction
// Order-preserving stream compaction of the mask into linear indices, in three passes over
// kScanChunk-cell blocks: per-block counts, one-block exclusive scan of the counts, per-block write.

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan of one value per thread over a block of kScanThreads; returns the block total in *total
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        before += (k < wid) ? wsum[k] : 0u;
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// the 16 mask bytes of a thread, [base, base + 16): one 16-byte load when all of them are in range and the
// address is 16-byte aligned (a lane per 16 bytes, so a wave reads 1 KiB contiguously), else byte by byte with
// the bytes past n read as 0
__device__ inline uint4 mask16(const uint8_t* __restrict__ mask, int64_t base, int64_t n) {
    static_assert(kScanPerThread == 16, "one 16-byte load per thread");
    if (base + 16 <= n && (reinterpret_cast<uintptr_t>(mask + base) & 15) == 0)
        return *reinterpret_cast<const uint4*>(mask + base);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int k = 0; k < 16; ++k)
        if (base + k < n) w[k >> 2] |= (uint32_t)mask[base + k] << (8 * (k & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// bit 7 of each byte of the result is set iff that byte of w is nonzero
__device__ inline uint32_t nonzero_bytes(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

__device__ inline uint32_t count16(const uint4 m) {
    return __popc(nonzero_bytes(m.x)) + __popc(nonzero_bytes(m.y)) + __popc(nonzero_bytes(m.z)) +
           __popc(nonzero_bytes(m.w));
}

__global__ __launch_bounds__(kScanThreads) void k_compact_count(const uint8_t* __restrict__ mask, int64_t n,
                                                                uint32_t* __restrict__ blk) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerThread;
    uint32_t total;
    (void)block_excl_scan(count16(mask16(mask, base, n)), &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// one block: exclusive scan of nb block counts in place; the grand total goes to *n_cells
__global__ __launch_bounds__(1024) void k_compact_scan(uint32_t* __restrict__ blk, int64_t nb,
                                                       int32_t* __restrict__ n_cells) {
    __shared__ uint32_t wsum[1024 / kWave];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    uint32_t local = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) local += blk[b0 + k];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(local);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int k = 0; k < 1024 / kWave; ++k) {
        before += (k < wid) ? wsum[k] : 0u;
        tot += wsum[k];
    }
    uint32_t run = before + inc - local;
    for (int64_t k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            const uint32_t v = blk[b0 + k];
            blk[b0 + k] = run;
            run += v;
        }
    }
    if (threadIdx.x == 0) *n_cells = (int32_t)tot;
}

__global__ __launch_bounds__(kScanThreads) void k_compact_write(const uint8_t* __restrict__ mask, int64_t n,
                                                                const uint32_t* __restrict__ blk,
                                                                int32_t* __restrict__ cells) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerThread;
    uint32_t total;
    const uint4 m = mask16(mask, base, n);
    uint32_t pos = blk[blockIdx.x] + block_excl_scan(count16(m), &total);
    const uint32_t w[4] = {nonzero_bytes(m.x), nonzero_bytes(m.y), nonzero_bytes(m.z), nonzero_bytes(m.w)};
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)  // bytes past n were read as 0
        if ((w[k >> 2] >> (8 * (k & 3) + 7)) & 1u) cells[pos++] = (int32_t)(base + k);
}

hipError_t launch_compact(const uint8_t* mask, int64_t n, int32_t* cells, int32_t* n_cells, uint32_t* blk,
                          hipStream_t s) {
    const int64_t nb = scan_blocks(n);
    if (nb == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)nb), dim3(kScanThreads), 0, s, mask, n, blk);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, blk, nb, n_cells);
    hipLaunchKernelGGL(k_compact_write, dim3((unsigned)nb), dim3(kScanThreads), 0, s, mask, n, blk, cells);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ raster helpers
// Fill kernels instead of memset nodes, so that the same sequence can be captured into a graph.
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 + 4 <= n && (reinterpret_cast<uintptr_t>(p + i0) & 15) == 0) {
        *reinterpret_cast<uint4*>(p + i0) = make_uint4(v, v, v, v);
    } else {
        for (int64_t i = i0; i < n && i < i0 + 4; ++i) p[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* __restrict__ p, unsigned long long v,
                                                  int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// DEM with a one-texel border replicating the edge texels: (H + 2) x (W + 2), row-major. Its texel
// (r + 1, c + 1) holds dem[clamp(r)][clamp(c)] for r in [-1, H], c in [-1, W], which is what the clamped
// bilinear patch reads, so the padded lookup needs no clamps.
__global__ __launch_bounds__(256) void k_pad_dem(const float* __restrict__ dem, int H, int W,
                                                 float* __restrict__ out) {
    // rows over blockIdx.y, columns over blockIdx.x and the threads: no division per texel
    const int64_t Wp = (int64_t)W + 2;
    for (int64_t rp = blockIdx.y; rp < (int64_t)H + 2; rp += gridDim.y) {
        const int64_t r = rp < 1 ? 0 : (rp > H ? H - 1 : rp - 1);
        const float* __restrict__ src = dem + r * W;
        float* __restrict__ dst = out + rp * Wp;
        for (int64_t cp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cp < Wp;
             cp += (int64_t)gridDim.x * blockDim.x) {
            const int64_t c = cp < 1 ? 0 : (cp > W ? W - 1 : cp - 1);
            dst[cp] = src[c];
        }
    }
}

// v^2 bits -> speed, in place: vmax = sqrt(max v^2)
__global__ __launch_bounds__(256) void k_finalize_vmax(uint32_t* __restrict__ bits, int64_t n) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 + 4 <= n && (reinterpret_cast<uintptr_t>(bits + i0) & 15) == 0) {
        uint4 b = *reinterpret_cast<uint4*>(bits + i0);
        b.x = __float_as_uint(sqrtf(__uint_as_float(b.x)));
        b.y = __float_as_uint(sqrtf(__uint_as_float(b.y)));
        b.z = __float_as_uint(sqrtf(__uint_as_float(b.z)));
        b.w = __float_as_uint(sqrtf(__uint_as_float(b.w)));
        *reinterpret_cast<uint4*>(bits + i0) = b;
    } else {
        for (int64_t i = i0; i < n && i < i0 + 4; ++i) bits[i] = __float_as_uint(sqrtf(__uint_as_float(bits[i])));
    }
}

static unsigned blocks_for(int64_t items, int per_thread) {
    const int64_t threads = (items + per_thread - 1) / per_thread;
    return (unsigned)((threads + 255) / 256);
}

hipError_t launch_pad_dem(const float* dem, int H, int W, float* out, hipStream_t s) {
    const int64_t col_blocks = std::min<int64_t>(((int64_t)W + 2 + 1023) / 1024, 1024);  // ~4 texels per thread
    const int64_t row_blocks = std::min<int64_t>((int64_t)H + 2, 65535);
    hipLaunchKernelGGL(k_pad_dem, dim3((unsigned)col_blocks, (unsigned)row_blocks), dim3(256), 0, s, dem, H, W, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 4)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 1)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ mipmap

// Up to kMipPass levels of the overlay mipmap in one pass. A block owns a 32 x 32 tile of the pass's
// first output level (a 64 x 64 tile of its input) and every coarser cell of that tile down to 1 x 1:
// each level halves the previous one rounding up, so the children of a cell never leave the tile.
// Counts add in 64 bits; speeds (>= 0) take the maximum; cells past a level's edge count as empty.
template <typename Tin>
__global__ __launch_bounds__(256) void k_mip(const Tin* __restrict__ cin, const float* __restrict__ vin, int h0, int w0,
                                             int nlev, MipLevels o) {
    __shared__ unsigned long long sc[32 * 32];
    __shared__ float sv[32 * 32];
    const int tr = blockIdx.y * 32, tc = blockIdx.x * 32;
    for (int k = threadIdx.x; k < 32 * 32; k += 256) {
        const int r = tr + k / 32, c = tc + k % 32;
        unsigned long long sum = 0;
        float mx = 0.0f;
        if (r < o.h[0] && c < o.w[0]) {
#pragma unroll
            for (int dr = 0; dr < 2; ++dr)
#pragma unroll
                for (int dc = 0; dc < 2; ++dc) {
                    const int rr = 2 * r + dr, cc = 2 * c + dc;
                    if (rr < h0 && cc < w0) {
                        const size_t i = (size_t)rr * w0 + cc;
                        sum += (unsigned long long)cin[i];
                        mx = fmaxf(mx, vin[i]);
                    }
                }
            o.c[0][(size_t)r * o.w[0] + c] = sum;
            o.v[0][(size_t)r * o.w[0] + c] = mx;
        }
        sc[k] = sum;
        sv[k] = mx;
    }
    __syncthreads();
    int side = 32;
    for (int l = 1; l < nlev; ++l) {
        const int s2 = side / 2;
        const int t = threadIdx.x;
        unsigned long long sum = 0;
        float mx = 0.0f;
        const int i = t / s2, j = t - (t / s2) * s2;
        if (t < s2 * s2) {
#pragma unroll
            for (int dr = 0; dr < 2; ++dr)
#pragma unroll
                for (int dc = 0; dc < 2; ++dc) {
                    sum += sc[(2 * i + dr) * side + 2 * j + dc];
                    mx = fmaxf(mx, sv[(2 * i + dr) * side + 2 * j + dc]);
                }
        }
        __syncthreads();
        if (t < s2 * s2) {
            sc[i * s2 + j] = sum;
            sv[i * s2 + j] = mx;
            const int r = blockIdx.y * s2 + i, c = blockIdx.x * s2 + j;
            if (r < o.h[l] && c < o.w[l]) {
                o.c[l][(size_t)r * o.w[l] + c] = sum;
                o.v[l][(size_t)r * o.w[l] + c] = mx;
            }
        }
        __syncthreads();
        side = s2;
    }
}

hipError_t launch_mip_pass(const void* cin, bool cin64, const float* vin, int h0, int w0, int nlev,
                           const MipLevels& o, hipStream_t s) {
    const dim3 grid((unsigned)((o.w[0] + 31) / 32), (unsigned)((o.h[0] + 31) / 32));
    if (cin64)
        hipLaunchKernelGGL(k_mip<unsigned long long>, grid, dim3(256), 0, s,
                           static_cast<const unsigned long long*>(cin), vin, h0, w0, nlev, o);
    else
        hipLaunchKernelGGL(k_mip<uint32_t>, grid, dim3(256), 0, s, static_cast<const uint32_t*>(cin), vin, h0, w0,
                           nlev, o);
    return hipGetLastError();
}

hipError_t launch_finalize_vmax(uint32_t* vmax_bits, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_vmax, dim3(blocks_for(n, 4)), dim3(256), 0, s, vmax_bits, n);
    return hipGetLastError();
}

}  // namespace avl
