// depth_sort.hip -- stable LSD radix sort of the per-Gaussian depth keys.
//
// The sort of Sec. 3.1 stage 3 orders (Gaussian, tile) pairs by the 64-bit
// key (tile << 32 | depth bits).  Every pair of one Gaussian carries the same
// 32 depth bits, so the least-significant digits of that LSD radix sort are
// applied here to the N Gaussians -- before duplication -- instead of to the
// K ~ 80 N pairs.  The tile digit is then one stable counting pass
// (tile_bin.hip) that writes each pair straight to its sorted position.
//
// Each 8-bit pass is reduce-then-scan: an LDS histogram per block, one
// exclusive scan of the digit-major [digit][block] table, and a stable
// scatter that ranks equal digits with wavefront ballots (lower lanes and
// earlier waves first).  Keys of Gaussians that overlap no tile are
// 0xFFFFFFFF and sink to the end; values start as the Gaussian index, so ties
// in depth stay in index order.
#include "gs_internal.h"

namespace gsmi {
namespace {

__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                 int shift, uint32_t* __restrict__ hist,
                                                                 int nblocks)
{
    __shared__ uint32_t h[4][256];   // one private histogram per wave
    const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
    for (int w = 0; w < 4; ++w) h[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + k * kSortBlock + tid;
        if (idx < n) atomicAdd(&h[wave][(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nblocks + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t n, int shift, const uint32_t* __restrict__ offsets, int nblocks)
{
    __shared__ uint32_t base[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base[tid] = offsets[(int64_t)tid * nblocks + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t blk = (int64_t)blockIdx.x * kSortTile;
    __syncthreads();
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = blk + k * kSortBlock + tid;
        const bool valid = idx < n;
        const uint32_t key = valid ? keys_in[idx] : 0u;
        const uint32_t val = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t cnt = (uint32_t)__popcll(m);
        uint32_t pos = 0;
        // waves take their offsets in order so equal digits keep input order
        for (int w = 0; w < 4; ++w) {
            if (wave == w && valid) {
                pos = base[d] + rank;
                if (rank == 0) base[d] = pos + cnt;
            }
            __syncthreads();
        }
        if (valid) {
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
    }
}

}  // namespace

size_t depth_sort_hist_elems(int64_t n)
{
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    return (size_t)(256 * (nb > 0 ? nb : 1));
}

// Sorts keys_in[0..n) (not modified) with values 0..n-1.  Four passes:
// in -> a -> b -> a -> b, so the sorted keys/values end in (keys_b, vals_b).
hipError_t launch_depth_sort(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                             uint32_t* vals_b, uint32_t* hist, uint64_t* scan_scratch, int64_t n, int* result_in_b,
                             hipStream_t s)
{
    *result_in_b = 1;
    if (n == 0) return hipSuccess;
    const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    uint32_t* kout = keys_a;
    uint32_t* vout = vals_a;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kSortBlock), 0, s, kin, n, shift, hist, nblocks);
        hipError_t e = launch_scan_exclusive(hist, (int64_t)256 * nblocks, scan_scratch, nullptr, nullptr, nullptr, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortBlock), 0, s, kin, vin, kout, vout, n,
                           shift, hist, nblocks);
        kin = kout;
        vin = vout;
        if (pass % 2 == 0) {
            kout = keys_b;
            vout = vals_b;
        } else {
            kout = keys_a;
            vout = vals_a;
        }
    }
    return hipGetLastError();
}

}  // namespace gsmi
