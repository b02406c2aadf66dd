// scan.hip -- device-wide exclusive prefix sum of uint32 values in two
// launches (tile sums, then a down-sweep in which every tile adds the sums of
// the tiles before it), used by the depth sort's digit offsets and by the
// binning's count arrays.  Tile sums and the total are
// accumulated in 64 bits; the total is written to *total (and an overflow
// flag raised when it does not fit 32 bits).  With n_dev set, the length is
// min(n, *n_dev), read on the device (no host sync).
#include "gs_internal.h"

namespace gsmi {
namespace {

constexpr int kScanThreads = 256;   // four waves (block_exclusive_u64)
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int64_t kScanMaxGrid = 8192;   // tiles beyond it are taken by grid-stride loops

__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t v, uint64_t* sh, uint64_t* total)
{
    // inclusive scan in each wave by shuffles, then the 4 wave totals in LDS
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (int w = 0; w < wave; ++w) before += sh[w];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();   // sh is reused by the next call
    return before + incl - v;
}

// LDS index of tile word e, one word of padding per 32 so that a thread's
// 16 consecutive words and a wave's 64 striped words spread over the banks
__device__ __forceinline__ int padded(int e) { return e + (e >> 5); }

__device__ __forceinline__ int64_t scan_length(int64_t n, const uint32_t* n_dev)
{
    if (!n_dev) return n;
    const int64_t d = (int64_t)*n_dev;
    return d < n ? d : n;
}

// Tiles of kScanTile values; the grid strides over the tiles of the device
// length (a grid sized for a bound then costs nothing past the real length).
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n_max,
                                                                    const uint32_t* n_dev,
                                                                    uint64_t* __restrict__ block_sums,
                                                                    const uint32_t* skip)
{
    if (skip && *skip) return;
    const int64_t n = scan_length(n_max, n_dev);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    __shared__ uint64_t sh[kScanThreads / 64];
    for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
        const int64_t base = t * kScanTile;
        // every load issued before any is used (a load under its own branch
        // is waited for before the next one issues); past n, word base (< n)
        // is loaded and dropped
        uint32_t x[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t i = base + k * kScanThreads + threadIdx.x;
            x[k] = in[i < n ? i : base];
        }
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k * kScanThreads + threadIdx.x < n) s += x[k];
        uint64_t tot;
        (void)block_exclusive_u64(s, sh, &tot);
        if (threadIdx.x == 0) block_sums[t] = tot;
    }
}

// exclusive scan of the tiles' sums by one block; writes the 64-bit total
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(uint64_t* __restrict__ sums, int64_t n_max,
                                                                   const uint32_t* n_dev, uint64_t* total_out,
                                                                   uint32_t* total32, uint32_t* overflow,
                                                                   const uint32_t* skip)
{
    if (skip && *skip) return;
    __shared__ uint64_t sh[kScanThreads / 64];
    const int64_t n = scan_length(n_max, n_dev);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t s = threadIdx.x * per, e = (s + per < nb) ? s + per : nb;
    uint64_t acc = 0;
    for (int64_t j = s; j < e; ++j) acc += sums[j];
    uint64_t tot;
    uint64_t run = block_exclusive_u64(acc, sh, &tot);
    for (int64_t j = s; j < e; ++j) {
        const uint64_t v = sums[j];
        sums[j] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        if (total_out) *total_out = tot;
        if (total32) *total32 = (uint32_t)tot;
        if (overflow && tot > 0xFFFFFFFFull) *overflow = 1u;
    }
}

// Down-sweep: every tile adds the sum of all tiles before it, computed by the
// block itself from the tile sums (there are at most a few thousand), so the
// scan needs no separate pass over the sums; the block of the last tile
// writes the total.
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(uint32_t* __restrict__ data, int64_t n_max,
                                                                 const uint32_t* n_dev,
                                                                 const uint64_t* __restrict__ tile_sums,
                                                                 uint64_t* total_out, uint32_t* total32,
                                                                 uint32_t* overflow, const uint32_t* skip)
{
    if (skip && *skip) return;
    const int64_t n = scan_length(n_max, n_dev);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    __shared__ uint64_t sh[kScanThreads / 64];
    __shared__ uint32_t s_tile[kScanTile + kScanTile / 32];
    if (nb == 0 && blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            if (total_out) *total_out = 0;
            if (total32) *total32 = 0;
        }
        return;
    }
    for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
        // prefix of the tile sums before t
        uint64_t p = 0;
        for (int64_t j = threadIdx.x; j < t; j += kScanThreads) p += tile_sums[j];
        uint64_t before;
        (void)block_exclusive_u64(p, sh, &before);
        const int64_t base = t * kScanTile;
        // thread i scans the kScanItems consecutive items [16 i, 16 i + 16) of
        // the tile; the tile moves between HBM and LDS in striped order
        // (consecutive lanes on consecutive words: whole cache lines) and is
        // regrouped in LDS
        uint32_t x[kScanItems];   // all loads first, as in scan_reduce_kernel
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t i = base + k * kScanThreads + threadIdx.x;
            x[k] = data[i < n ? i : base];
        }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int e = k * kScanThreads + threadIdx.x;
            s_tile[padded(e)] = (base + e < n) ? x[k] : 0u;
        }
        __syncthreads();
        uint32_t v[kScanItems];
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = s_tile[padded(threadIdx.x * kScanItems + k)];
            s += v[k];
        }
        uint64_t tot;
        uint64_t run = block_exclusive_u64(s, sh, &tot) + before;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            s_tile[padded(threadIdx.x * kScanItems + k)] = (uint32_t)run;
            run += v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int e = k * kScanThreads + threadIdx.x;
            if (base + e < n) data[base + e] = s_tile[padded(e)];
        }
        __syncthreads();   // s_tile is reused by the next tile
        if (t == nb - 1 && threadIdx.x == 0) {
            const uint64_t total = before + tot;
            if (total_out) *total_out = total;
            if (total32) *total32 = (uint32_t)total;
            if (overflow && total > 0xFFFFFFFFull) *overflow = 1u;
        }
    }
}

}  // namespace

size_t scan_scratch_elems(int64_t n)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb > 0 ? nb : 1);
}

hipError_t launch_scan_exclusive(uint32_t* data, int64_t n, uint64_t* block_scratch, uint64_t* total64,
                                 uint32_t* total32, uint32_t* overflow, hipStream_t s, const uint32_t* n_dev,
                                 const uint32_t* skip)
{
    if (n <= 0) {
        if (total64 || total32) {
            hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, block_scratch, (int64_t)0,
                               (const uint32_t*)nullptr, total64, total32, overflow, skip);
        }
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    const unsigned grid = (unsigned)std::min<int64_t>(nb, kScanMaxGrid);
    // one tile: the down-sweep reads no tile sums (none precede tile 0)
    if (nb > 1)
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(grid), dim3(kScanThreads), 0, s, data, n, n_dev, block_scratch,
                           skip);
    hipLaunchKernelGGL(scan_down_kernel, dim3(grid), dim3(kScanThreads), 0, s, data, n, n_dev, block_scratch,
                       total64, total32, overflow, skip);
    return hipGetLastError();
}

}  // namespace gsmi
