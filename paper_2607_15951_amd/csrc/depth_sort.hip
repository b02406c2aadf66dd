// depth_sort.hip -- stable LSD radix sort of the per-Gaussian depth keys.
//
// The sort of Sec. 3.1 stage 3 orders (Gaussian, tile) pairs by the 64-bit
// key (tile << 32 | depth bits).  Every pair of one Gaussian carries the same
// 32 depth bits, so the least-significant digits of that LSD radix sort are
// applied here to the N Gaussians -- before duplication -- instead of to the
// K ~ 80 N pairs.  The tile digit is then one stable counting pass
// (tile_bin.hip) that writes each pair straight to its sorted position.
//
// Several views are sorted at once as segments of one array (one segment per
// view, items v * n + i); no block straddles two segments.
//
// Each 8-bit pass is reduce-then-scan: an LDS histogram per block, one
// exclusive scan of the digit-major [segment][digit][block] table, and a stable
// scatter that ranks equal digits with wavefront ballots (lower lanes and
// earlier waves first).  Keys of Gaussians that overlap no tile are
// 0xFFFFFFFF and sink to the end; values start as the Gaussian index, so ties
// in depth stay in index order.
#include "gs_internal.h"

namespace gsmi {
namespace {

// Block b sorts part lb = b % bpv of segment v = b / bpv: items
// [v * n + lb * tile, min(.. + tile, (v + 1) * n)), tile = kSortBlock * kItems.
// The digit table is [segment][digit][part], so its exclusive scan keeps the
// segments apart and stable within each.
template <int kItems>
__device__ __forceinline__ void sort_block_range(int64_t n, int bpv, int64_t* begin, int64_t* end, int64_t* row)
{
    constexpr int64_t tile = (int64_t)kSortBlock * kItems;
    const int v = (int)(blockIdx.x / (unsigned)bpv), lb = (int)(blockIdx.x % (unsigned)bpv);
    *begin = (int64_t)v * n + (int64_t)lb * tile;
    const int64_t seg_end = (int64_t)(v + 1) * n;
    *end = (*begin + tile < seg_end) ? *begin + tile : seg_end;
    *row = (int64_t)v * 256 * bpv + lb;   // table index of digit 0; digit d adds d * bpv
}

template <int kItems>
__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                 int shift, uint32_t* __restrict__ hist, int bpv)
{
    __shared__ uint32_t h[4][256];   // one private histogram per wave
    const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
    for (int w = 0; w < 4; ++w) h[w][tid] = 0;
    __syncthreads();
    int64_t begin, end, row;
    sort_block_range<kItems>(n, bpv, &begin, &end, &row);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kSortBlock + tid;
        if (idx < end) atomicAdd(&h[wave][(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[row + (int64_t)tid * bpv] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

// Stable scatter of one block's items.  Item (round k, wave w, lane l) is
// idx = begin + k * kSortBlock + 64 w + l, so the input order is (k, w, l).
// Each wave ranks its items of a round among equal digits with eight ballots
// (lanes holding the same digit) and records the group's size in
// cnt[k][w][d]; one pass of 256 threads (one per digit) turns those counts
// into exclusive offsets in (k, w) order, and every item lands at
// base[d] + cnt[k][w][d] + (lanes of its group below it) -- two barriers per
// block instead of a hand-over per (round, wave).
template <int kItems>
__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t n, int shift, const uint32_t* __restrict__ offsets, int bpv)
{
    __shared__ uint32_t cnt[kItems][4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t begin, end, row;
    sort_block_range<kItems>(n, bpv, &begin, &end, &row);
    for (int k = 0; k < kItems; ++k)
        for (int w = 0; w < 4; ++w) cnt[k][w][tid] = 0u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
    uint32_t key[kItems], val[kItems], digit[kItems], rank[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kSortBlock + tid;
        const bool valid = idx < end;
        key[k] = valid ? keys_in[idx] : 0u;
        val[k] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (key[k] >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        digit[k] = valid ? d : 256u;
        rank[k] = (uint32_t)__popcll(m & lt);
        // the group's first lane records its size (groups are disjoint)
        if (valid && rank[k] == 0) cnt[k][wave][d] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    {   // thread d: exclusive prefix of digit d over (round, wave), plus the block's base
        uint32_t run = offsets[row + (int64_t)tid * bpv];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = cnt[k][w][tid];
                cnt[k][w][tid] = run;
                run += c;
            }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (digit[k] < 256u) {
            const uint32_t pos = cnt[k][wave][digit[k]] + rank[k];
            keys_out[pos] = key[k];
            vals_out[pos] = val[k];
        }
    }
}

template <int kItems>
void launch_sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint32_t* hist,
                      int64_t n, int shift, int bpv, unsigned nblocks, bool histogram_only, hipStream_t s)
{
    if (histogram_only)
        hipLaunchKernelGGL(radix_hist_kernel<kItems>, dim3(nblocks), dim3(kSortBlock), 0, s, kin, n, shift, hist, bpv);
    else
        hipLaunchKernelGGL(radix_scatter_kernel<kItems>, dim3(nblocks), dim3(kSortBlock), 0, s, kin, vin, kout, vout,
                           n, shift, hist, bpv);
}

}  // namespace

bool depth_sort_items_supported(int items) { return items == 4 || items == 8 || items == 16; }

size_t depth_sort_hist_elems(int64_t n, int n_views)
{
    // sized for the smallest block (the most blocks) any supported width uses
    const int64_t tile = (int64_t)kSortBlock * 4;
    const int64_t bpv = (n + tile - 1) / tile;
    const int64_t nb = bpv * (n_views > 0 ? n_views : 1);
    return (size_t)(256 * (nb > 0 ? nb : 1));
}

// Sorts each of the n_views segments keys_in[v * n .. (v + 1) * n) (not
// modified) with values v * n + i, items keys per thread of a block.  Four
// passes: in -> a -> b -> a -> b, so the sorted keys/values end in (keys_b,
// vals_b).
hipError_t launch_depth_sort(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                             uint32_t* vals_b, uint32_t* hist, uint64_t* scan_scratch, int64_t n, int n_views,
                             int items, int* result_in_b, hipStream_t s)
{
    *result_in_b = 1;
    if (n == 0 || n_views <= 0) return hipSuccess;
    if (!depth_sort_items_supported(items)) return hipErrorInvalidValue;
    const int64_t tile = (int64_t)kSortBlock * items;
    const int bpv = (int)((n + tile - 1) / tile);
    const unsigned nblocks = (unsigned)bpv * (unsigned)n_views;
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    uint32_t* kout = keys_a;
    uint32_t* vout = vals_a;
    auto pass_launch = [&](int shift, bool hist_only) {
        switch (items) {
        case 4: launch_sort_pass<4>(kin, vin, kout, vout, hist, n, shift, bpv, nblocks, hist_only, s); break;
        case 8: launch_sort_pass<8>(kin, vin, kout, vout, hist, n, shift, bpv, nblocks, hist_only, s); break;
        default: launch_sort_pass<16>(kin, vin, kout, vout, hist, n, shift, bpv, nblocks, hist_only, s); break;
        }
    };
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        pass_launch(shift, true);
        hipError_t e = launch_scan_exclusive(hist, (int64_t)256 * nblocks, scan_scratch, nullptr, nullptr, nullptr, s);
        if (e != hipSuccess) return e;
        pass_launch(shift, false);
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
