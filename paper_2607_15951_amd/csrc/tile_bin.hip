// tile_bin.hip -- duplication of Gaussians into (tile, depth) pairs fused with
// the stable tile-digit pass of the key sort.
//
// Every Gaussian overlapping a screen tile (the 3-sigma square of Sec. 4.4)
// yields one pair; a pair's key is (tile << 32 | depth bits), its value the
// Gaussian index.  Gaussians arrive here already in (depth, index) order
// (depth_sort.hip), so a stable counting sort on the tile digit leaves every
// tile's list in front-to-back order: the output IS the sorted pair list.
//
// Work decomposition: one wavefront per (chunk of kBinChunk consecutive
// depth-sorted Gaussians, band of tile rows with <= kMaxBandTiles tiles).  A
// wave expands its Gaussians' rectangles, clipped to its band, into a flat
// sequence of pairs (Gaussian-major, then tile row, then column) and walks it
// 64 pairs at a time, so large and small Gaussians share lanes evenly.
//   count:   LDS histogram per (chunk, band) -> counts[chunk][tile]
//   offsets: exclusive scan over chunks per tile, then over tiles
//   scatter: per (chunk, band) LDS cursors start at tile offset + chunk
//            prefix; equal tiles within a 64-pair group are ranked by lane
//            (ballot match on the tile bits), which keeps Gaussian order.
#include "gs_internal.h"

namespace gsmi {
namespace {

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Shared walk over the pairs of one (chunk, band); calls emit(local_tile,
// gaussian, active) once per 64-pair group with every lane of the wave.
template <class Emit>
__device__ __forceinline__ void walk_pairs(const BinArgs& a, int chunk, int ty0, int ty1, Emit&& emit)
{
    __shared__ uint32_t s_incl[64];
    __shared__ int s_x0[64], s_w[64], s_row0[64];
    __shared__ uint32_t s_g[64];
    const int lane = threadIdx.x;
    const int64_t nv = (int64_t)*a.n_visible;
    const int64_t start = (int64_t)chunk * kBinChunk;
    const int64_t end = (start + kBinChunk < nv) ? start + kBinChunk : nv;
    for (int64_t base = start; base < end; base += 64) {
        const int64_t pos = base + lane;
        uint32_t mine = 0, g = 0;
        int x0 = 0, w = 1, row0 = 0;
        if (pos < end) {
            g = a.sorted_idx[pos];
            const ushort4 r = a.rect[g];
            const int y0 = (int)r.y > ty0 ? (int)r.y : ty0;
            const int y1 = (int)r.w < ty1 ? (int)r.w : ty1;
            if (y1 > y0) {
                x0 = r.x;
                w = (int)r.z - (int)r.x;
                row0 = y0 - ty0;
                mine = (uint32_t)(w * (y1 - y0));
            }
        }
        const uint32_t incl = wave_inclusive_scan(mine, lane);
        const uint32_t total = __shfl(incl, 63, 64);
        s_incl[lane] = incl;
        s_x0[lane] = x0;
        s_w[lane] = w;
        s_row0[lane] = row0;
        s_g[lane] = g;
        __syncthreads();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + lane;
            const bool active = p < total;
            int local = 0;
            uint32_t gi = 0;
            if (active) {
                int lo = 0, hi = 63;   // first lane whose inclusive count exceeds p
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_incl[mid] > p) hi = mid; else lo = mid + 1;
                }
                const uint32_t j = p - (lo ? s_incl[lo - 1] : 0u);
                const uint32_t ws = (uint32_t)s_w[lo];
                const uint32_t row = j / ws;
                const uint32_t col = j - row * ws;
                local = (s_row0[lo] + (int)row) * a.tiles_x + s_x0[lo] + (int)col;
                gi = s_g[lo];
            }
            emit(local, gi, active);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void bin_count_kernel(BinArgs a)
{
    __shared__ uint32_t cnt[kMaxBandTiles];
    const int chunk = blockIdx.x, band = blockIdx.y, lane = threadIdx.x;
    const int ty0 = band * a.band_rows;
    const int ty1 = (ty0 + a.band_rows < a.tiles_y) ? ty0 + a.band_rows : a.tiles_y;
    const int band_tiles = (ty1 - ty0) * a.tiles_x;
    for (int k = lane; k < band_tiles; k += 64) cnt[k] = 0;
    __syncthreads();
    walk_pairs(a, chunk, ty0, ty1, [&](int local, uint32_t, bool active) {
        if (active) atomicAdd(&cnt[local], 1u);
    });
    __syncthreads();
    const int64_t T = (int64_t)a.tiles_x * a.tiles_y;
    uint32_t* dst = a.counts + (int64_t)chunk * T + (int64_t)ty0 * a.tiles_x;
    for (int k = lane; k < band_tiles; k += 64) dst[k] = cnt[k];
}

// counts[c][t] -> exclusive prefix over c (in place); totals[t] = column sum.
// Block: 64 tiles x 16 chunk segments.
__global__ __launch_bounds__(1024) void bin_colscan_kernel(uint32_t* __restrict__ counts, int C, int T,
                                                           uint32_t* __restrict__ totals)
{
    __shared__ uint32_t part[16][64];
    const int tl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + tl;
    const int per = (C + 15) / 16;
    const int c0 = seg * per, c1 = (c0 + per < C) ? c0 + per : C;
    uint32_t s = 0;
    if (t < T)
        for (int c = c0; c < c1; ++c) s += counts[(int64_t)c * T + t];
    part[seg][tl] = s;
    __syncthreads();
    uint32_t run = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
        const uint32_t v = part[k][tl];
        if (k < seg) run += v;
        tot += v;
    }
    if (t < T) {
        for (int c = c0; c < c1; ++c) {
            const int64_t o = (int64_t)c * T + t;
            const uint32_t v = counts[o];
            counts[o] = run;
            run += v;
        }
        if (seg == 0) totals[t] = tot;
    }
}

// tile_offsets[t] = sum of totals[<t]; tile_offsets[T] = K (u32), and K in
// 64 bits at *k_total.  Flags overflow when K does not fit the capacity or
// 32 bits.  One 1024-thread block.
__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t* __restrict__ totals, int T,
                                                         uint32_t* __restrict__ offsets, uint64_t* k_total,
                                                         uint64_t capacity, uint32_t* overflow)
{
    __shared__ uint64_t part[1024];
    const int tid = threadIdx.x;
    const int per = (T + 1023) / 1024;
    const int s = tid * per, e = (s + per < T) ? s + per : T;
    uint64_t sum = 0;
    for (int j = s; j < e; ++j) sum += totals[j];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - sum;
    for (int j = s; j < e; ++j) {
        offsets[j] = (uint32_t)run;
        run += totals[j];
    }
    if (tid == 1023) {
        const uint64_t K = part[1023];
        offsets[T] = (uint32_t)K;
        *k_total = K;
        if (K > capacity || K > 0xFFFFFFFFull) *overflow = 1u;
    }
}

__global__ __launch_bounds__(64) void bin_scatter_kernel(BinArgs a)
{
    __shared__ uint32_t cursor[kMaxBandTiles];
    const int chunk = blockIdx.x, band = blockIdx.y, lane = threadIdx.x;
    const int ty0 = band * a.band_rows;
    const int ty1 = (ty0 + a.band_rows < a.tiles_y) ? ty0 + a.band_rows : a.tiles_y;
    const int band_tiles = (ty1 - ty0) * a.tiles_x;
    const int64_t T = (int64_t)a.tiles_x * a.tiles_y;
    const uint32_t* prefix = a.counts + (int64_t)chunk * T + (int64_t)ty0 * a.tiles_x;
    const uint32_t* toff = a.tile_offsets + (int64_t)ty0 * a.tiles_x;
    for (int k = lane; k < band_tiles; k += 64) cursor[k] = toff[k] + prefix[k];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t cap = a.capacity;
    uint32_t* values = a.values;
    walk_pairs(a, chunk, ty0, ty1, [&](int local, uint32_t g, bool active) {
        const uint64_t act = __ballot(active);
        if (!active) return;
        uint64_t m = act;
#pragma unroll
        for (int b = 0; b < 11; ++b) {   // kMaxBandTiles = 2^11
            const bool bit = (local >> b) & 1;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t first = cursor[local];
        const uint32_t pos = first + rank;
        if (rank == 0) cursor[local] = first + (uint32_t)__popcll(m);
        if ((uint64_t)pos < cap) values[pos] = g;
    });
}

}  // namespace

hipError_t launch_bin_count(const BinArgs& a, hipStream_t s)
{
    if (a.num_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_count_kernel, dim3(a.num_chunks, a.num_bands), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_offsets(const BinArgs& a, hipStream_t s, uint64_t* k_total)
{
    const int T = a.tiles_x * a.tiles_y;
    if (a.num_chunks > 0)
        hipLaunchKernelGGL(bin_colscan_kernel, dim3((T + 63) / 64), dim3(1024), 0, s, a.counts, a.num_chunks, T,
                           a.totals);
    else
        (void)launch_fill_u32(a.totals, 0u, T, s);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, s, a.totals, T, a.tile_offsets, k_total,
                       a.capacity, a.overflow);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const BinArgs& a, hipStream_t s)
{
    if (a.num_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(a.num_chunks, a.num_bands), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsmi
