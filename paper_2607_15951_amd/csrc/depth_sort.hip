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
// Each 8-bit pass is reduce-then-scan in three launches: an LDS histogram
// per block, written as the block's 256 contiguous counts (whole cache
// lines; a digit-major table would take 256 scattered partial-line writes
// per block); one workgroup per (segment, digit) that gathers its digit's
// counts over the blocks, scans them into the digit-major
// [segment][digit][block] offset table and records the digit's total; and a
// stable scatter that ranks equal digits with wavefront ballots (lower lanes
// and earlier waves first) and places digit d of segment v at v * n +
// (totals of the smaller digits) + (its row's exclusive prefix).  Digits are taken from sort_key(key), which orders
// depths as numbers (negative ones, behind the camera, first); keys of
// Gaussians without a finite depth are 0xFFFFFFFF and sink to the end.
// Values start as the Gaussian index, so ties in depth stay in index order.
// A segment that fits one block takes one launch per pass: the scatter
// counts its block's digits itself (no histogram, no offset table).
#include "gs_internal.h"

namespace gsmi {
namespace {

// Block b sorts part lb = b % bpv of segment v = b / bpv: items
// [v * n + lb * tile, min(.. + tile, (v + 1) * n)), tile = kSortBlock * kItems.
// The count buffer holds the digit totals [segment][digit], the offset
// table [segment][digit][part], then the block histograms [block][digit].
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

// Order-preserving map of a depth key to the sort key: float bits compare as
// unsigned integers only among non-negative floats, so negative depths
// (Gaussians behind the camera) are flipped below them; 0xFFFFFFFF (no finite
// depth) stays last.  On the non-negative depths of the pairs it keeps the
// order of the bits themselves.
__device__ __forceinline__ uint32_t sort_key(uint32_t b)
{
    if (b == 0xFFFFFFFFu) return b;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

template <int kItems>
__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                 int shift, uint32_t* __restrict__ hist, int bpv,
                                                                 const uint32_t* skip)
{
    if (skip && *skip) return;   // the previous frame's order was reused
    __shared__ uint32_t h[4][256];   // one private histogram per wave
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int w = 0; w < 4; ++w) h[w][tid] = 0;
    __syncthreads();
    int64_t begin, end, row;
    sort_block_range<kItems>(n, bpv, &begin, &end, &row);
    // every key load issued before any is used (a load under its own branch
    // is waited for before the next one issues); past end, key begin is
    // loaded and dropped
    uint32_t kk[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kSortBlock + tid;
        kk[k] = keys[idx < end ? idx : begin];
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kSortBlock + tid;
        const bool valid = idx < end;
        const uint32_t d = valid ? (sort_key(kk[k]) >> shift) & 255u : 0u;
        const uint64_t m = __ballot(valid);
        if (m == 0) continue;
        // the high digits of nearby depths are mostly one value: a wave whose
        // items share it counts them with one atomic instead of 64 colliding
        const int first = __ffsll((long long)m) - 1;
        const uint32_t d0 = (uint32_t)__shfl((int)d, first, 64);
        if (__ballot(valid && d != d0) == 0) {
            if (lane == first) atomicAdd(&h[wave][d0], (uint32_t)__popcll(m));
        } else if (valid) {
            atomicAdd(&h[wave][d], 1u);
        }
    }
    __syncthreads();
    (void)row;   // the histogram goes to the block's own row of 256 counts, not to the offset table
    hist[(int64_t)blockIdx.x * 256 + tid] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

// Workgroup (v, d): exclusive scan of digit d's counts over the bpv blocks of
// segment v (hist[(v * bpv + b) * 256 + d]) into row (v, d) of the offset
// table, and the digit's total in totals[v * 256 + d].  Counts fit 32 bits
// (n_views * n < 2^32).
constexpr int kScanRowItems = 8;
__global__ __launch_bounds__(256) void radix_row_scan_kernel(const uint32_t* __restrict__ hist,
                                                              uint32_t* __restrict__ table,
                                                              uint32_t* __restrict__ totals, int bpv,
                                                              const uint32_t* skip)
{
    if (skip && *skip) return;
    __shared__ uint32_t s_wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int v = (int)(blockIdx.x >> 8), d = (int)(blockIdx.x & 255u);
    const uint32_t* col = hist + (int64_t)v * bpv * 256 + d;   // block b's count at col[b * 256]
    uint32_t* row = table + (int64_t)blockIdx.x * bpv;
    uint32_t carry = 0u;
    for (int base = 0; base < bpv; base += 256 * kScanRowItems) {
        uint32_t x[kScanRowItems], run = 0u;
        const int j0 = base + tid * kScanRowItems;   // this thread's consecutive counts
#pragma unroll
        for (int k = 0; k < kScanRowItems; ++k) {
            x[k] = (j0 + k < bpv) ? col[(int64_t)(j0 + k) * 256] : 0u;
            run += x[k];
        }
        uint32_t incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += s_wsum[w];
        const uint32_t chunk_total = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
        uint32_t acc = before + incl - run;
#pragma unroll
        for (int k = 0; k < kScanRowItems; ++k) {
            if (j0 + k < bpv) row[j0 + k] = acc;
            acc += x[k];
        }
        carry += chunk_total;
        __syncthreads();   // s_wsum is reused by the next chunk
    }
    if (tid == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one block's items.  Item (round k, wave w, lane l) is
// idx = begin + k * kSortBlock + 64 w + l, so the input order is (k, w, l).
// Each wave ranks its items of a round among equal digits with eight ballots
// (lanes holding the same digit) and records the group's size in
// cnt[k][w][d]; one pass of 256 threads (one per digit) turns those counts
// into exclusive offsets in (k, w) order and the digits' totals into the
// block's digit starts.  Every item is then placed in LDS at its position in
// the block's stable digit order, and the block writes that order out with
// consecutive threads on consecutive positions of each digit's run: item i of
// digit d goes to base[d] + (i - start[d]).  The global writes come as whole
// runs instead of one scattered word per lane.
//
// With kPay every item also carries a payload word: read from pay_in, or in
// the first pass (pay_in null) packed from rect_in, and written to pay_out
// beside its value.  keys_out may be null (the last pass: the sorted keys
// are not needed).
template <int kItems, bool kPay, int kThreads = kSortBlock>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const ushort4* __restrict__ rect_in, const uint32_t* __restrict__ pay_in,
    uint32_t* __restrict__ pay_out, int64_t n, int shift, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ totals, int bpv, const uint32_t* skip)
{
    constexpr int kWaves = kThreads / 64;
    constexpr int kBlockItems = kItems * kThreads;   // = kSortBlock * (kBlockItems / kSortBlock): the block's part
    static_assert(kThreads % kSortBlock == 0, "whole 256-thread groups");
    if (skip && *skip) return;
    // the block's keys, values (and payloads) in digit order; before that,
    // the 16-bit ranking counts cnt[k][w][d] (at most kBlockItems)
    // in the same bytes, which keeps the block's LDS at 8 (12) bytes per item
    __shared__ uint32_t s_buf[(kPay ? 3 : 2) * kBlockItems];
    uint16_t(*cnt)[kWaves][256] = reinterpret_cast<uint16_t(*)[kWaves][256]>(s_buf);
    static_assert(kItems * kWaves * 256 * sizeof(uint16_t) <= sizeof(s_buf), "ranking counts fit the key buffer");
    static_assert(kBlockItems <= 65535, "16-bit ranking offsets");
    __shared__ uint32_t s_start[256], s_base[256], s_wsum[4], s_ssum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t begin, end, row;
    sort_block_range<kBlockItems / kSortBlock>(n, bpv, &begin, &end, &row);
    for (int i = tid; i < kItems * kWaves * 128; i += kThreads) s_buf[i] = 0u;   // cnt, two counts per word
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
    uint32_t key[kItems], val[kItems], digit[kItems], rank[kItems];
    uint32_t pay[kPay ? kItems : 1];
    // all loads first (see radix_hist_kernel)
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kThreads + tid;
        const int64_t ic = idx < end ? idx : begin;
        key[k] = keys_in[ic];
        val[k] = vals_in ? vals_in[ic] : (uint32_t)idx;
        if constexpr (kPay) pay[k] = pay_in ? pay_in[ic] : pack_rect(rect_in[ic]);
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t idx = begin + k * kThreads + tid;
        const bool valid = idx < end;
        if (!valid) key[k] = val[k] = 0u;
        const uint32_t d = (sort_key(key[k]) >> shift) & 255u;
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
        if (valid && rank[k] == 0) cnt[k][wave][d] = (uint16_t)__popcll(m);
    }
    __syncthreads();
    // threads d < 256: exclusive offsets of digit d over (round, wave), its
    // total, and the block's digit start (exclusive prefix of the totals);
    // then the segment's start of digit d (exclusive prefix of its totals)
    const int v = (int)(blockIdx.x / (unsigned)bpv);
    uint32_t run = 0u, seg_total = 0u, incl = 0u, seg_incl = 0u;
    if (tid < 256) {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = cnt[k][w][tid];
                cnt[k][w][tid] = (uint16_t)run;
                run += c;
            }
        // the segment's count of digit d: from the digit totals, or, when the
        // block is the whole segment (no totals), the block's own count
        seg_total = totals ? totals[v * 256 + tid] : run;
        incl = run;
        seg_incl = seg_total;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64), u = __shfl_up(seg_incl, o, 64);
            if (lane >= o) {
                incl += t;
                seg_incl += u;
            }
        }
        if (lane == 63) {
            s_wsum[wave] = incl;
            s_ssum[wave] = seg_incl;
        }
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t before = 0u, seg_before = (uint32_t)((int64_t)v * n);
        for (int w = 0; w < wave; ++w) {
            before += s_wsum[w];
            seg_before += s_ssum[w];
        }
        s_start[tid] = before + incl - run;
        s_base[tid] = seg_before + seg_incl - seg_total + (offsets ? offsets[row + (int64_t)tid * bpv] : 0u);
    }
    __syncthreads();
    uint32_t local[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        local[k] = digit[k] < 256u ? s_start[digit[k]] + cnt[k][wave][digit[k]] + rank[k] : ~0u;
    __syncthreads();   // cnt is reused below
    uint32_t* s_key = s_buf;
    uint32_t* s_val = s_key + kBlockItems;
    uint32_t* s_pay = s_val + kBlockItems;   // kPay only
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (local[k] != ~0u) {
            s_key[local[k]] = key[k];
            s_val[local[k]] = val[k];
            if constexpr (kPay) s_pay[local[k]] = pay[k];
        }
    }
    __syncthreads();
    const int count = (int)(end - begin);
    for (int i = tid; i < count; i += kThreads) {
        const uint32_t kk = s_key[i];
        const uint32_t d = (sort_key(kk) >> shift) & 255u;
        const uint32_t pos = s_base[d] + ((uint32_t)i - s_start[d]);
        if (keys_out) keys_out[pos] = kk;
        vals_out[pos] = s_val[i];
        if constexpr (kPay) pay_out[pos] = s_pay[i];
    }
}

// One 8-bit pass: histogram, row scans, scatter.  counts = totals
// [n_views][256], the offset table [n_views][256][bpv], the block
// histograms [nblocks][256].
template <int kItems>
void launch_sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const ushort4* rect,
                      const uint32_t* pin, uint32_t* pout, uint32_t* counts, int64_t n, int n_views, int shift,
                      int bpv, unsigned nblocks, const uint32_t* skip, hipStream_t s)
{
    uint32_t* totals = counts;
    uint32_t* table = counts + (int64_t)256 * n_views;
    uint32_t* hist = table + (int64_t)256 * nblocks;
    if (bpv > 1) {
        hipLaunchKernelGGL(radix_hist_kernel<kItems>, dim3(nblocks), dim3(kSortBlock), 0, s, kin, n, shift, hist,
                           bpv, skip);
        hipLaunchKernelGGL(radix_row_scan_kernel, dim3(256u * (unsigned)n_views), dim3(256), 0, s,
                           (const uint32_t*)hist, table, totals, bpv, skip);
    } else {
        // one block per segment: the scatter counts the digits itself
        totals = table = nullptr;
    }
    // the scatter of a 16-key part runs as 1024 threads of 4 keys: the same
    // part, ranked by 16 waves of 4 rounds instead of 4 waves of 16 (0.161
    // against 0.165 ms for the four passes at 3M keys; parts of 8192 keys,
    // one 100 KB block per CU, took 0.20 ms)
    constexpr int kThreads = kItems == 16 ? 1024 : kSortBlock;
    constexpr int kPer = kItems * kSortBlock / kThreads;
    if (pout)
        hipLaunchKernelGGL((radix_scatter_kernel<kPer, true, kThreads>), dim3(nblocks), dim3(kThreads), 0, s, kin, vin,
                           kout, vout, rect, pin, pout, n, shift, (const uint32_t*)table, (const uint32_t*)totals, bpv,
                           skip);
    else
        hipLaunchKernelGGL((radix_scatter_kernel<kPer, false, kThreads>), dim3(nblocks), dim3(kThreads), 0, s, kin,
                           vin, kout, vout, rect, pin, pout, n, shift, (const uint32_t*)table, (const uint32_t*)totals,
                           bpv, skip);
}

// ------------------------------------------------- reuse of the previous order
// Between nearby frames few Gaussians change their tile (the data locality of
// Sec. 5.7, Table 5), but their depth order is another matter: a dense scene
// has depth gaps far below the depth change of a small camera step, so most
// adjacent pairs swap.  The previous frame's order (one view, same Gaussians)
// is therefore only tried, and cheaply: each item gets this frame's key in
// that order and the descents (adjacent pairs out of order) are counted.
//   no descent       the order holds (static camera, appearance-only
//                    changes): the radix passes are skipped;
//   a few descents   runs of kReuseBlock items are sorted in LDS twice
//                    (aligned, then shifted by half a run) and the result is
//                    checked; the passes are skipped if it holds;
//   more             the radix passes sort from scratch.
// Every decision is taken on the device (flags the kernels read), so the
// frame needs no host read and can be captured.  Whatever path runs, the
// order is the stable (depth, index) order: the check compares the composite
// (sort key << 32 | index), a strict total order.
constexpr int kReuseThreads = 1024;
constexpr int kReuseItems = 8;
constexpr int kReuseBlock = kReuseThreads * kReuseItems;   // items sorted together in LDS

// The gathered keys are sort keys (sort_key), as the radix passes compare.
// words[0] = 1 while the reused order holds (the radix passes' skip flag),
// words[1] = descents of the gathered previous order (churn), words[2] = 1
// when the local repair runs.  A repair is tried for at most n / kRepairFraction descents.
constexpr int64_t kRepairFraction = 256;
// One item per thread: item j takes this frame's key of prev[j], and each
// block counts its descents (pairs (j, j + 1) out of order, the pair across
// its end included) into partial[block].  No counter is shared: one atomic
// counter hit by every block serialises when most pairs swap.  The successor
// of lane l is lane l + 1's item; lane 63 loads its own.
__global__ __launch_bounds__(256) void order_gather_kernel(const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ prev, int64_t n,
                                                           uint32_t* __restrict__ k_out, uint32_t* __restrict__ v_out,
                                                           uint32_t* words, uint32_t* __restrict__ partial)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool in = j < n;
    uint32_t p = prev[in ? j : 0];
    const bool tail = lane == 63 && j + 1 < n;
    uint32_t p1 = tail ? prev[j + 1] : 0u;
    const bool invalid = in && p >= (uint32_t)n;   // not an order of these items: sort from scratch
    p = p < (uint32_t)n ? p : 0u;
    p1 = p1 < (uint32_t)n ? p1 : 0u;
    const uint32_t k = sort_key(keys[p]);
    const uint32_t k1 = tail ? sort_key(keys[p1]) : 0u;
    if (in) {
        k_out[j] = k;
        v_out[j] = p;
    }
    uint32_t kn = __shfl_down(k, 1, 64), pn = __shfl_down(p, 1, 64);
    if (lane == 63) {
        kn = k1;
        pn = p1;
    }
    const uint64_t cur = ((uint64_t)k << 32) | p, next = ((uint64_t)kn << 32) | pn;
    uint32_t descents = (j + 1 < n && cur > next) ? 1u : 0u;
    if (invalid) words[0] = 0u;
    __shared__ uint32_t s_d[4];
    for (int o = 32; o > 0; o >>= 1) descents += __shfl_xor(descents, o, 64);
    if (lane == 0) s_d[threadIdx.x >> 6] = descents;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = s_d[0] + s_d[1] + s_d[2] + s_d[3];
}

// Sorts runs of kReuseBlock composite keys in LDS (bitonic network).  Run b
// covers [offset + b * kReuseBlock, ...); with kShifted the runs start half a
// run in, and one extra block copies the first half run unchanged.
// (The unshifted pass sorts in place: in and out may be the same arrays.)
template <bool kShifted>
__global__ __launch_bounds__(kReuseThreads) void order_local_sort_kernel(const uint32_t* k_in, const uint32_t* v_in,
                                                                        int64_t n, uint32_t* k_out, uint32_t* v_out,
                                                                        const uint32_t* words)
{
    if (!words[2]) return;   // no repair this frame
    __shared__ uint64_t s[kReuseBlock];
    const int tid = threadIdx.x;
    const int64_t half = kReuseBlock / 2;
    if (kShifted && blockIdx.x == gridDim.x - 1) {   // the head, already in place
        for (int64_t i = tid; i < half && i < n; i += kReuseThreads) {
            k_out[i] = k_in[i];
            v_out[i] = v_in[i];
        }
        return;
    }
    const int64_t base = (kShifted ? half : 0) + (int64_t)blockIdx.x * kReuseBlock;
#pragma unroll
    for (int k = 0; k < kReuseItems; ++k) {
        const int64_t i = base + k * kReuseThreads + tid;
        s[k * kReuseThreads + tid] = i < n ? (((uint64_t)k_in[i] << 32) | v_in[i]) : ~0ull;   // pads sort last
    }
    __syncthreads();
    for (int size = 2; size <= kReuseBlock; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int k = 0; k < kReuseBlock / 2 / kReuseThreads; ++k) {
                const int c = k * kReuseThreads + tid;   // pair index
                const int lo = 2 * stride * (c / stride) + (c % stride), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = s[lo], b = s[hi];
                if ((a > b) == up) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < kReuseItems; ++k) {
        const int64_t i = base + k * kReuseThreads + tid;
        if (i < n) {
            const uint64_t c = s[k * kReuseThreads + tid];
            k_out[i] = (uint32_t)(c >> 32);
            v_out[i] = (uint32_t)c;
        }
    }
}

// After the gather: no descent keeps the order as it is (the previous order
// in vals_b is this frame's order), a few start the repair, more give up.
__global__ __launch_bounds__(1024) void order_plan_kernel(uint32_t* words, const uint32_t* __restrict__ partial,
                                                           int blocks, int64_t n)
{
    // the descents: the gather blocks' counts summed
    __shared__ unsigned long long s_sum[16];
    unsigned long long t = 0;
    for (int b = threadIdx.x; b < blocks; b += 1024) t += partial[b];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long total = 0;
    for (int w = 0; w < 16; ++w) total += s_sum[w];
    const uint32_t d = (uint32_t)total;   // at most n - 1 < 2^32
    words[1] = d;
    const bool valid = words[0] != 0u;
    const bool repair = valid && d > 0u && (int64_t)d <= n / kRepairFraction;
    words[2] = repair ? 1u : 0u;
    words[0] = (valid && (d == 0u || repair)) ? 1u : 0u;
}

// Clears words[0] at any descent left after the two local sorts.
__global__ __launch_bounds__(256) void order_check_kernel(const uint32_t* __restrict__ k, const uint32_t* __restrict__ v,
                                                          int64_t n, uint32_t* words)
{
    if (!words[2]) return;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j + 1 < n) {
        const uint64_t a = ((uint64_t)k[j] << 32) | v[j], b = ((uint64_t)k[j + 1] << 32) | v[j + 1];
        if (a > b) words[0] = 0u;
    }
}

// The rectangles in a reused order (see launch_order_pack).
__global__ __launch_bounds__(256) void order_pack_kernel(const uint32_t* __restrict__ order,
                                                         const ushort4* __restrict__ rect, int64_t n,
                                                         const uint32_t* words, uint32_t* __restrict__ pay)
{
    if (!words[0]) return;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) pay[j] = pack_rect(rect[order[j]]);
}

}  // namespace

hipError_t launch_order_pack(const uint32_t* vals_b, const ushort4* rect, int64_t n, const uint32_t* words,
                             uint32_t* pay_b, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vals_b, rect, n, words,
                       pay_b);
    return hipGetLastError();
}

bool depth_sort_items_supported(int items) { return items == 4 || items == 8 || items == 16; }

size_t order_reuse_words(int64_t n) { return (size_t)(kReuseWords + (n + 255) / 256); }

size_t depth_sort_hist_elems(int64_t n, int n_views)
{
    // digit totals, then the offset table and the block histograms, both
    // sized for the smallest block (the most blocks) any supported width uses
    const int64_t tile = (int64_t)kSortBlock * 4;
    const int64_t bpv = (n + tile - 1) / tile;
    const int64_t V = n_views > 0 ? n_views : 1;
    const int64_t nb = bpv * V;
    return (size_t)(256 * (V + 2 * (nb > 0 ? nb : 1)));
}

hipError_t launch_order_reuse(const uint32_t* keys, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                              uint32_t* vals_b, int64_t n, uint32_t* words, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_fill_u32(words, 0u, kReuseWords, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(words, 1u, 1, s);
    if (e != hipSuccess) return e;
    const unsigned g256 = (unsigned)((n + 255) / 256);
    // previous order (vals_b) -> (this frame's keys, items) in a
    uint32_t* partial = words + kReuseWords;
    hipLaunchKernelGGL(order_gather_kernel, dim3(g256), dim3(256), 0, s, keys, (const uint32_t*)vals_b, n, keys_a,
                       vals_a, words, partial);
    hipLaunchKernelGGL(order_plan_kernel, dim3(1), dim3(1024), 0, s, words, (const uint32_t*)partial, (int)g256, n);
    const int64_t half = kReuseBlock / 2;
    const unsigned runs = (unsigned)((n + kReuseBlock - 1) / kReuseBlock);
    const unsigned runs_shifted = (unsigned)(n > half ? (n - half + kReuseBlock - 1) / kReuseBlock : 0) + 1u;
    hipLaunchKernelGGL(order_local_sort_kernel<false>, dim3(runs), dim3(kReuseThreads), 0, s, (const uint32_t*)keys_a,
                       (const uint32_t*)vals_a, n, keys_a, vals_a, (const uint32_t*)words);
    hipLaunchKernelGGL(order_local_sort_kernel<true>, dim3(runs_shifted), dim3(kReuseThreads), 0, s,
                       (const uint32_t*)keys_a, (const uint32_t*)vals_a, n, keys_b, vals_b, (const uint32_t*)words);
    hipLaunchKernelGGL(order_check_kernel, dim3(g256), dim3(256), 0, s, (const uint32_t*)keys_b, (const uint32_t*)vals_b,
                       n, words);
    return hipGetLastError();
}

// Sorts each of the n_views segments keys_in[v * n .. (v + 1) * n) (not
// modified) with values v * n + i, items keys per thread of a block.  Four
// passes: in -> a -> b -> a -> b, so the sorted values (and payloads) end in
// vals_b (pay_b); the last pass writes no keys.  With reuse_words (one view,
// after launch_order_reuse) every pass reads words[0] on the device and does
// nothing when the reused order holds.
hipError_t launch_depth_sort(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                             uint32_t* vals_b, const ushort4* rect, uint32_t* pay_a, uint32_t* pay_b,
                             uint32_t* counts, int64_t n, int n_views, int items, const uint32_t* reuse_words,
                             hipStream_t s)
{
    if (n == 0 || n_views <= 0) return hipSuccess;
    if (!depth_sort_items_supported(items)) return hipErrorInvalidValue;
    const int64_t tile = (int64_t)kSortBlock * items;
    const int bpv = (int)((n + tile - 1) / tile);
    const unsigned nblocks = (unsigned)bpv * (unsigned)n_views;
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    const uint32_t* pin = nullptr;   // the first pass packs from rect
    const uint32_t* skip = reuse_words;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        const bool to_b = pass % 2 == 1;
        uint32_t* kout = pass == 3 ? nullptr : (to_b ? keys_b : keys_a);
        uint32_t* vout = to_b ? vals_b : vals_a;
        uint32_t* pout = rect ? (to_b ? pay_b : pay_a) : nullptr;
        switch (items) {
        case 4: launch_sort_pass<4>(kin, vin, kout, vout, rect, pin, pout, counts, n, n_views, shift, bpv, nblocks, skip, s); break;
        case 8: launch_sort_pass<8>(kin, vin, kout, vout, rect, pin, pout, counts, n, n_views, shift, bpv, nblocks, skip, s); break;
        default: launch_sort_pass<16>(kin, vin, kout, vout, rect, pin, pout, counts, n, n_views, shift, bpv, nblocks, skip, s); break;
        }
        kin = kout;
        vin = vout;
        pin = pout;
    }
    return hipGetLastError();
}

}  // namespace gsmi
