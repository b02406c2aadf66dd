// tile_bin.hip -- duplication of Gaussians into (tile, depth) pairs fused with
// the stable tile-digit pass of the key sort.
//
// Every Gaussian overlapping a screen tile (the 3-sigma square of Sec. 4.4)
// yields one pair; a pair's key is (tile << 32 | depth bits), its value the
// Gaussian index.  Gaussians arrive here in (depth, index) order
// (depth_sort.hip), so a stable distribution on the tile digit leaves every
// tile's list in front-to-back order: the output IS the sorted pair list.
//
// The tile digit is distributed in two stable levels:
//   level 1  every depth-sorted Gaussian is copied to the list of each tile
//            row its rectangle spans: row entries (index, x0 | x1 << 16);
//   level 2  every row entry is copied to the list of each tile of that row
//            its column span covers: the pair values.
// A wavefront owns a chunk of consecutive items (Gaussians, or one row's
// entries), kept in registers, a few per lane (the autotuner picks how many).  It walks the buckets
// (rows, or the row's tile columns) in order; for bucket x every item of a
// batch of 64 tests whether its span covers x, M = ballot(covers), and the
// covering lanes write at cursor[x] + (number of covering lanes below them),
// after which cursor[x] advances by popcount(M).  Items keep their order
// inside every bucket, each bucket's run is written front to back, and the
// work is one compare per (item, bucket) -- no per-pair search or ranking.
//   count    per chunk, an LDS difference array (+1 at a span's first bucket,
//            -1 past its last), summed into per-bucket counts, stored
//            bucket-major: count[bucket][chunk];
//   scan     one device-wide exclusive scan of that array: entry
//            [bucket][chunk] becomes the chunk's cursor in the bucket, i.e.
//            the bucket's list offset plus the items of earlier chunks;
//   scatter  the walk from those cursors.
#include "gs_internal.h"

#include <type_traits>

namespace gsmi {
namespace {

constexpr int kBand = 8;                 // tile columns per band of the level-2 walk (8: measured fastest of 4 to 32)

// info[] layout (uint32): [0] level-2 chunks C2, [1] level-2 count elements
// E2, then for the global tile rows r = 0..rows: [kInfoRowChunks + r] level-2
// chunk prefix, [kInfoRowChunks + rows + 1 + r] count-element prefix.  Row r
// owns chunks(r) = prefix[r + 1] - prefix[r] chunks and the count elements
// [eprefix[r], eprefix[r] + tiles_x(r) * chunks(r)), bucket-major:
// count[x * chunks(r) + j].
constexpr int kInfoRowChunks = 2;

__device__ __forceinline__ const uint32_t* row_chunk_prefix(const BinArgs& a) { return a.info + kInfoRowChunks; }
__device__ __forceinline__ const uint32_t* row_elem_prefix(const BinArgs& a)
{
    return a.info + kInfoRowChunks + a.rows + 1;
}

// Workgroup b -> chunk: the dispatcher deals workgroups round-robin to the 8
// XCDs; block b takes chunk (b % 8) * ceil(grid / 8) + b / 8 so each XCD works
// through a contiguous run of chunks, whose output pieces are adjacent.
__device__ __forceinline__ int chunk_of_block()
{
    const int per_xcd = (int)((gridDim.x + 7) / 8);
    return (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
}

// Number of covering lanes below this one in mask m (lanes 0..lane-1).
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int t = __shfl_xor(v, o, 64);
        v = t < v ? t : v;
    }
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

// ------------------------------------------------------------------ level 1
// items: depth-sorted Gaussians of one view; buckets: that view's tile rows;
// payload (item, x-span).  Level-1 chunk c belongs to view c / chunks1 and is
// part c % chunks1 of that view's keyed items (which open its segment; those
// culled or off screen have an empty rectangle).

template <int kItems>
struct Items1 {
    // rows [y0, y0 + h) covered (rows of the view); h = 0 for padding lanes
    uint32_t y0[kItems], h[kItems], xs[kItems], g[kItems];
    int lo, hi;        // rows spanned by the chunk
    int view, part;    // view, chunk index within the view
};

// Keyed-item range [start, end) of level-1 chunk c; false when empty.
__device__ __forceinline__ bool chunk1_range(const BinArgs& a, int c, int* view, int* part, int64_t* start,
                                             int64_t* end)
{
    *view = c / a.chunks1;
    *part = c % a.chunks1;
    if (*view >= a.n_views) return false;
    const int64_t seg = (int64_t)(*view) * a.n;
    // the view's keyed items (finite depth) open its segment; the culled or
    // off-screen ones among them have an empty rectangle and yield no entry
    const int64_t nv = (int64_t)a.view_counts[(int64_t)kViewCounters * (*view) + 1];
    *start = seg + (int64_t)(*part) * (a.items1 * 64);
    *end = seg + nv;
    return *start < *end;
}

template <int kItems>
__device__ __forceinline__ bool load_items1(const BinArgs& a, int c, int lane, Items1<kItems>& it)
{
    int64_t start, end;
    if (!chunk1_range(a, c, &it.view, &it.part, &start, &end)) return false;
    int lo = 1 << 30, hi = 0;
#pragma unroll
    for (int b = 0; b < kItems; ++b) {
        const int64_t k = start + b * 64 + lane;
        ushort4 r = make_ushort4(0, 0, 0, 0);
        uint32_t g = 0;
        if (k < end) {
            g = a.sorted_idx[k];
            r = a.sorted_pack ? unpack_rect(a.sorted_pack[k]) : a.sorted_rect[k];
            if (r.w > r.y) {   // an off-screen item spans no row
                lo = (int)r.y < lo ? (int)r.y : lo;
                hi = (int)r.w > hi ? (int)r.w : hi;
            }
        }
        it.y0[b] = r.y;
        it.h[b] = (uint32_t)r.w - (uint32_t)r.y;
        it.xs[b] = (uint32_t)r.x | ((uint32_t)r.z << 16);
        it.g[b] = g;
    }
    it.lo = __builtin_amdgcn_readfirstlane(wave_min(lo));   // uniform: keep it scalar
    it.hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    return true;
}

// Difference arrays in LDS are kept in kDiffCopies interleaved copies, bucket
// x of copy c at x * kDiffCopies + c, and lane l adds to copy l % kDiffCopies:
// lanes that hit the same bucket mostly hit different words, so the atomics
// of a wave collide less.
constexpr int kDiffCopies = 4;
__device__ __forceinline__ uint32_t* diff_slot(uint32_t* diff, uint32_t x, int lane)
{
    return diff + x * kDiffCopies + (lane & (kDiffCopies - 1));
}
__device__ __forceinline__ uint32_t diff_at(const uint32_t* diff, int x)
{
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < kDiffCopies; ++c) v += diff[x * kDiffCopies + c];
    return v;
}

// Exclusive-then-inclusive sum of a difference array diff[0..m) (LDS) by one
// wave: dst[x * stride] = diff[0] + ... + diff[x], the count of spans covering x.
__device__ __forceinline__ void counts_from_diff(const uint32_t* diff, int m, uint32_t* dst, int64_t stride,
                                                 int lane)
{
    const int per = (m + 63) / 64;
    const int b = lane * per, e = (b + per < m) ? b + per : m;
    uint32_t s = 0;
    for (int k = b; k < e; ++k) s += diff_at(diff, k);
    uint32_t run = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(run, o, 64);
        if (lane >= o) run += t;
    }
    run -= s;
    for (int k = b; k < e; ++k) {
        run += diff_at(diff, k);
        dst[k * stride] = run;
    }
}

// Counting needs no order: each span adds +1 at its first bucket and -1 past
// its last in an LDS difference array (two atomics per item), summed at the end.
template <int kItems>
__global__ __launch_bounds__(64) void level1_count_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    extern __shared__ uint32_t diff[];   // [max_tiles_y + 1][kDiffCopies], sized at launch
    const int lane = threadIdx.x, c = chunk_of_block();
    const int view = c / a.chunks1, part = c % a.chunks1;
    if (view >= a.n_views) return;
    const ViewParams& vp = a.views[view];
    for (int r = lane; r < (vp.tiles_y + 1) * kDiffCopies; r += 64) diff[r] = 0u;
    __syncthreads();
    int v2, p2;
    int64_t start = 0, end = 0;
    (void)chunk1_range(a, c, &v2, &p2, &start, &end);
    if (a.sorted_pack) {
        // the rectangles in depth order, carried there by the sort: read in
        // order, all loads before any counting
        uint32_t pk[kItems];
#pragma unroll
        for (int b = 0; b < kItems; ++b) {
            const int64_t k = start + b * 64 + lane;
            pk[b] = k < end ? a.sorted_pack[k] : 0u;
        }
#pragma unroll
        for (int b = 0; b < kItems; ++b) {
            const ushort4 r = unpack_rect(pk[b]);   // empty for lanes past the end
            if (r.w > r.y) {
                atomicAdd(diff_slot(diff, r.y, lane), 1u);
                atomicSub(diff_slot(diff, r.w, lane), 1u);
            }
        }
    } else {
        // the rectangles gathered in depth order, for the scatter to stream:
        // all index loads, then all gathers, then the counting (see
        // load_items2)
        uint32_t idx[kItems];
#pragma unroll
        for (int b = 0; b < kItems; ++b) {
            const int64_t k = start + b * 64 + lane;
            idx[b] = k < end ? a.sorted_idx[k] : 0u;
        }
        ushort4 rr[kItems];
#pragma unroll
        for (int b = 0; b < kItems; ++b) rr[b] = a.rect[idx[b]];
#pragma unroll
        for (int b = 0; b < kItems; ++b) {
            const int64_t k = start + b * 64 + lane;
            if (k < end) {
                const ushort4 r = rr[b];
                a.sorted_rect[k] = r;
                if (r.w > r.y) {
                    atomicAdd(diff_slot(diff, r.y, lane), 1u);
                    atomicSub(diff_slot(diff, r.w, lane), 1u);
                }
            }
        }
    }
    __syncthreads();
    counts_from_diff(diff, vp.tiles_y, a.counts1 + (int64_t)vp.row_base * a.chunks1 + part, a.chunks1, lane);
}

// The row walk goes band by band (kRowBand rows): the chunk's items that
// reach band b are packed, in chunk order, into dense batches in LDS (payload
// and their rows inside the band), and only those batches walk the band's
// rows.  An item covers a few of the view's rows, so a plain walk of every
// row against every batch would mostly test items that miss the row.  Inside
// a row the items keep their chunk order, so the output is that of the plain
// walk.  Cursors of a band's rows are loaded into one VGPR (lane q: row
// b0 + q) and read back as scalars.
constexpr int kRowBand = 8;   // measured: 4 and 12 were slower
static_assert(kRowBand <= 15, "band-relative rows in 4 bits");

template <bool kChecked>
__device__ __forceinline__ void walk_row_band(const uint2* s_p, const uint8_t* s_r, uint32_t n, uint32_t cur_b,
                                              uint2* __restrict__ out, uint64_t capacity, int lane)
{
    uint32_t cur[kRowBand];
#pragma unroll
    for (int q = 0; q < kRowBand; ++q) cur[q] = __builtin_amdgcn_readlane(cur_b, q);
    for (uint32_t k0 = 0; k0 < n; k0 += 64) {
        const uint32_t k = k0 + lane;
        uint32_t rs = 0u;
        uint2 p = make_uint2(0u, 0u);
        if (k < n) {
            rs = s_r[k];
            p = s_p[k];
        }
        // band-relative rows [r0, r0 + w): packed items are clipped to the
        // band and to the view, so a row outside them is never covered
        const uint32_t r0 = rs & 15u, w = (rs >> 4) - r0;
#pragma unroll
        for (int q = 0; q < kRowBand; ++q) {
            const bool cover = (uint32_t)q - r0 < w;
            const uint64_t m = __ballot(cover);
            if (cover) {
                const uint32_t pos = cur[q] + lanes_below(m);
                if (!kChecked || pos < capacity) out[pos] = p;
            }
            cur[q] += (uint32_t)__popcll(m);
        }
    }
}

template <int kItems>
__global__ __launch_bounds__(64) void level1_scatter_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    __shared__ uint2 s_p[kItems * 64];
    __shared__ uint8_t s_r[kItems * 64];
    const int lane = threadIdx.x, c = chunk_of_block();
    Items1<kItems> it;
    if (!load_items1(a, c, lane, it)) return;
    // row r of the view: cursor[r * chunks1]
    const uint32_t* cursor = a.counts1 + (int64_t)a.views[it.view].row_base * a.chunks1 + it.part;
    auto band_cursors = [&](int b0) -> uint32_t {
        const int r = b0 + lane;
        return (lane < kRowBand && r < it.hi) ? cursor[(int64_t)r * a.chunks1] : 0u;
    };
    const int blo = it.lo / kRowBand * kRowBand;
    uint32_t cur_b = blo < it.hi ? band_cursors(blo) : 0u;
    for (int b0 = blo; b0 < it.hi; b0 += kRowBand) {
        const uint32_t by0 = (uint32_t)b0, by1 = min((uint32_t)(b0 + kRowBand), (uint32_t)it.hi);
        const uint32_t cur_next = (b0 + kRowBand < it.hi) ? band_cursors(b0 + kRowBand) : 0u;   // prefetch
        // pack the items reaching the band, clipped to it, in chunk order
        uint32_t n = 0;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t e0 = max(it.y0[j], by0), e1 = min(it.y0[j] + it.h[j], by1);
            const bool reach = e1 > e0;
            const uint64_t m = __ballot(reach);
            if (reach) {
                const uint32_t slot = n + lanes_below(m);
                s_p[slot] = make_uint2(it.g[j], it.xs[j]);
                s_r[slot] = (uint8_t)((e0 - by0) | ((e1 - by0) << 4));   // 0 <= e0 < e1 <= kRowBand
            }
            n += (uint32_t)__popcll(m);
        }
        __syncthreads();
        // row cursors increase down the view: the band's last one bounds them all
        const uint32_t cur_last = __builtin_amdgcn_readlane(cur_b, (int)(by1 - by0) - 1);
        if ((uint64_t)cur_last + n <= a.row_capacity)
            walk_row_band<false>(s_p, s_r, n, cur_b, a.row_ent, a.row_capacity, lane);
        else
            walk_row_band<true>(s_p, s_r, n, cur_b, a.row_ent, a.row_capacity, lane);
        __syncthreads();   // the LDS is free for the next band
        cur_b = cur_next;
    }
}

// Row offsets and the level-2 chunk table (one 1024-thread block, a run of
// ceil(rows / 1024) rows per thread, so a few rows take one step each).  The scanned level-1 counts give rows_off[r] (chunk 0's
// cursor in row r); row r owns ceil(len_r / chunk2) level-2 chunks (chunk2 =
// 64 items2 entries) and
// tiles_x(r) count elements per chunk; info holds both prefixes.  On
// overflow every row gets zero chunks.
static_assert(kMaxTotalRows % 1024 == 0, "rows per thread of the chunk table");

__global__ __launch_bounds__(1024) void level2_table_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    __shared__ uint32_t wave_c[16], wave_e[16];
    __shared__ uint32_t s_total_c, s_total_e;
    const int tid = threadIdx.x, rows = a.rows, lane = tid & 63, wave = tid >> 6;
    const uint32_t chunk2 = (uint32_t)a.items2 * 64u;
    const int per = (rows + 1023) / 1024;   // at most kMaxTotalRows / 1024
    const int r0 = tid * per;
    for (int k = 0; k < per; ++k) {
        const int r = r0 + k;
        if (r < rows) a.rows_off[r] = a.counts1[(int64_t)r * a.chunks1];
    }
    __syncthreads();   // rows_off[rows] (= R) was written by the scan
    uint32_t sc = 0, se = 0;
    for (int k = 0; k < per; ++k) {
        const int r = r0 + k;
        if (r < rows) {
            const uint32_t len = a.rows_off[r + 1] - a.rows_off[r];
            const uint32_t ch = (len + chunk2 - 1) / chunk2;
            sc += ch;
            se += ch * a.row_tiles_x[r];
        }
    }
    // inclusive prefixes over the threads: in the wave, then over the waves
    uint32_t ic = sc, ie = se;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t tc = __shfl_up(ic, o, 64), te = __shfl_up(ie, o, 64);
        if (lane >= o) {
            ic += tc;
            ie += te;
        }
    }
    if (lane == 63) {
        wave_c[wave] = ic;
        wave_e[wave] = ie;
    }
    __syncthreads();
    for (int w = 0; w < wave; ++w) {
        ic += wave_c[w];
        ie += wave_e[w];
    }
    if (tid == 1023) {
        uint32_t tc = ic, te = ie;
        if ((int64_t)tc > (int64_t)a.max_chunks2 || (uint64_t)te > a.counts2_capacity ||
            (uint64_t)a.rows_off[rows] > a.row_capacity) {
            *a.overflow = 1u;
            tc = te = 0;
        }
        s_total_c = tc;
        s_total_e = te;
    }
    __syncthreads();
    const bool ok = s_total_c != 0u;
    uint32_t run_c = ok ? ic - sc : 0u, run_e = ok ? ie - se : 0u;
    uint32_t* cpre = a.info + kInfoRowChunks;
    uint32_t* epre = a.info + kInfoRowChunks + rows + 1;
    for (int k = 0; k < per; ++k) {
        const int r = r0 + k;
        if (r < rows) {
            cpre[r] = run_c;
            epre[r] = run_e;
            if (ok) {
                const uint32_t ch = (a.rows_off[r + 1] - a.rows_off[r] + chunk2 - 1) / chunk2;
                run_c += ch;
                run_e += ch * a.row_tiles_x[r];
            }
        }
    }
    if (tid == 0) {
        cpre[rows] = s_total_c;
        epre[rows] = s_total_e;
        a.info[kInfoC2] = s_total_c;
        a.info[kInfoC2Elems] = s_total_e;
    }
}

// ------------------------------------------------------------------ level 2
// items: one row's entries; buckets: that row's tile columns; payload: index

template <int kItems>
struct Items2 {
    // columns [x0, x1) covered, packed x0 | x1 << 16; empty for padding lanes
    uint32_t xs[kItems], g[kItems];
    int row, lo, hi;   // row, columns spanned by the chunk
    const uint32_t* cursor;   // column x's cursor at cursor[x * stride]
    int64_t stride;           // the row's level-2 chunks
};

// Start of chunk c's cursors in the scanned level-2 counts: row r's block
// starts at eprefix[r], column x at x * chunks(r), chunk c at c - prefix[r].
__device__ __forceinline__ const uint32_t* level2_slot(const BinArgs& a, int row, int c, int64_t* stride)
{
    const uint32_t* base = row_chunk_prefix(a);
    *stride = (int64_t)(base[row + 1] - base[row]);
    return a.counts2 + (int64_t)row_elem_prefix(a)[row] + (c - (int64_t)base[row]);
}

// Row and entry range [eb, ee) of level-2 chunk c.
__device__ __forceinline__ void chunk2_range(const BinArgs& a, int c, int lane, int* row, int64_t* eb, int64_t* ee)
{
    const int rows = a.rows;
    const uint32_t* base = row_chunk_prefix(a);
    // owning row: the last r with base[r] <= c (64-ary search over rows; rows
    // without chunks share base with the next row, so the last one owns c)
    int L = 0, R = rows;
    while (R - L > 1) {
        const int step = (R - L + 63) / 64;
        const int q = L + lane * step;
        const bool ok = q < R && base[q] <= (uint32_t)c;
        const uint64_t m = __ballot(ok);
        const int top = 63 - (int)__clzll((long long)m);
        const int nl = L + top * step;
        R = (nl + step < R) ? nl + step : R;
        L = nl;
    }
    *row = __builtin_amdgcn_readfirstlane(L);
    const int64_t chunk2 = (int64_t)a.items2 * 64;
    *eb = (int64_t)a.rows_off[*row] + (int64_t)((uint32_t)c - base[*row]) * chunk2;
    const int64_t end_row = a.rows_off[*row + 1];
    *ee = (*eb + chunk2 < end_row) ? *eb + chunk2 : end_row;
}

template <int kItems>
__device__ __forceinline__ bool load_items2(const BinArgs& a, int c, int lane, Items2<kItems>& it)
{
    if ((uint32_t)c >= a.info[kInfoC2]) return false;
    int64_t eb, ee;
    chunk2_range(a, c, lane, &it.row, &eb, &ee);
    // every load is issued before any is used (a load under its own branch
    // would be waited for before the next is issued); lanes past the chunk
    // load entry eb, which exists, and drop it
    uint2 ent[kItems];
#pragma unroll
    for (int b = 0; b < kItems; ++b) {
        const int64_t e = eb + b * 64 + lane;
        ent[b] = a.row_ent[e < ee ? e : eb];
    }
    int lo = 1 << 30, hi = 0;
#pragma unroll
    for (int b = 0; b < kItems; ++b) {
        const bool in = eb + b * 64 + lane < ee;
        const uint32_t xs = in ? ent[b].y : 0u;
        if (in) {
            const int x0 = (int)(xs & 0xFFFFu), x1 = (int)(xs >> 16);
            lo = x0 < lo ? x0 : lo;
            hi = x1 > hi ? x1 : hi;
        }
        it.xs[b] = xs;
        it.g[b] = in ? ent[b].x : 0u;
    }
    it.lo = __builtin_amdgcn_readfirstlane(wave_min(lo));   // uniform: keep it scalar
    it.hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    it.cursor = level2_slot(a, it.row, c, &it.stride);
    return true;
}

// One level-2 chunk's per-column counts.
template <int kItems>
__device__ __forceinline__ void level2_count_chunk(const BinArgs& a, int c, int lane, uint32_t* diff)
{
    int row;
    int64_t eb, ee;
    chunk2_range(a, c, lane, &row, &eb, &ee);
    const int row_tx = (int)a.row_tiles_x[row];
    for (int x = lane; x < (row_tx + 1) * kDiffCopies; x += 64) diff[x] = 0u;
    __syncthreads();
    // all loads first (see load_items2), then the counting
    uint32_t xs[kItems];
#pragma unroll
    for (int b = 0; b < kItems; ++b) {
        const int64_t e = eb + b * 64 + lane;
        xs[b] = a.row_ent[e < ee ? e : eb].y;
    }
#pragma unroll
    for (int b = 0; b < kItems; ++b) {
        if (eb + b * 64 + lane < ee) {
            atomicAdd(diff_slot(diff, xs[b] & 0xFFFFu, lane), 1u);
            atomicSub(diff_slot(diff, xs[b] >> 16, lane), 1u);
        }
    }
    __syncthreads();
    int64_t stride;
    uint32_t* dst = const_cast<uint32_t*>(level2_slot(a, row, c, &stride));
    counts_from_diff(diff, row_tx, dst, stride, lane);
    __syncthreads();   // diff is reused by the next chunk
}

// The level-2 kernels stride over the device's chunk count c2, so a grid
// sized for a bound (pair_capacity mode) costs nothing past the real chunks.
// XCD x (blocks b with b % 8 == x, as the dispatcher deals them) owns the
// contiguous run of chunks [x * per, (x + 1) * per), per = ceil(c2 / 8), and
// its blocks take them in turn: every XCD has a share of the work whatever
// the grid, and each XCD's output pieces are adjacent.  (With the grid of
// an eager render, 8 ceil(c2 / 8) blocks, each block takes one chunk.)
#define FOR_LEVEL2_CHUNK(c, c2)                                                        \
    for (int per_ = ((c2) + 7) / 8, j_ = (int)(blockIdx.x >> 3), c = (int)(blockIdx.x & 7) * per_ + j_; \
         j_ < per_ && c < (c2); j_ += (int)(gridDim.x >> 3), c += (int)(gridDim.x >> 3))

template <int kItems>
__global__ __launch_bounds__(64) void level2_count_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    extern __shared__ uint32_t diff[];   // [max_tiles_x + 1][kDiffCopies], sized at launch: more waves fit
    const int lane = threadIdx.x;
    const int c2 = (int)a.info[kInfoC2];
    FOR_LEVEL2_CHUNK(c, c2) level2_count_chunk<kItems>(a, c, lane, diff);
}

// The walk of one band over the n packed entries in LDS (s_g, s_x): batch
// by batch, each batch against the band's kBand columns, unrolled so that
// every column's cursor stays in a scalar register.  cur_b holds the cursors
// (lane q: column bx0 + q).
template <bool kChecked>
__device__ __forceinline__ void walk_band(const uint32_t* s_g, const uint16_t* s_x, uint32_t n, uint32_t bx0,
                                          uint32_t cur_b, uint32_t* __restrict__ out, uint64_t capacity, int lane)
{
    uint32_t cur[kBand];
#pragma unroll
    for (int q = 0; q < kBand; ++q) cur[q] = __builtin_amdgcn_readlane(cur_b, q);
    for (uint32_t k0 = 0; k0 < n; k0 += 64) {
        const uint32_t k = k0 + lane;
        uint32_t xs = 0u, g = 0u;
        if (k < n) {
            xs = s_x[k];
            g = s_g[k];
        }
        // band-relative span [x0, x0 + w): packed entries are clipped to the
        // band and to the image, so a column outside them is never covered
        const uint32_t x0 = xs & 31u, w = (xs >> 5) - x0;
#pragma unroll
        for (int q = 0; q < kBand; ++q) {
            const bool cover = (uint32_t)q - x0 < w;
            const uint64_t m = __ballot(cover);
            if (cover) {
                const uint32_t pos = cur[q] + lanes_below(m);
                if (!kChecked || pos < capacity) out[pos] = g;
            }
            cur[q] += (uint32_t)__popcll(m);
        }
    }
}

// A plain walk would test every batch of the chunk against every column the
// chunk spans (about the row width), while an entry covers a few columns.
// The chunk is walked band by band instead (kBand columns): the entries that
// reach band b are packed, in chunk order, into dense batches through LDS,
// and only those batches walk the band's columns.  Inside a column the
// entries keep their chunk order, so the output is that of the plain walk.
template <int kItems>
__device__ __forceinline__ void level2_scatter_chunk(const BinArgs& a, int c, int lane, uint32_t* s_g, uint16_t* s_x)
{
    Items2<kItems> it;
    if (!load_items2(a, c, lane, it)) return;
    const int blo = it.lo / kBand, bhi = (it.hi + kBand - 1) / kBand;
    const int row_tx = (int)a.row_tiles_x[it.row];
    // cursors of band b's columns: lane l < kBand holds column b * kBand + l
    auto band_cursors = [&](int b) -> uint32_t {
        const int col = b * kBand + lane;
        return (lane < kBand && col < row_tx) ? it.cursor[col * it.stride] : 0u;
    };
    uint32_t cur_b = band_cursors(blo);
    for (int b = blo; b < bhi; ++b) {
        const uint32_t bx0 = (uint32_t)(b * kBand), bx1 = min(bx0 + kBand, (uint32_t)row_tx);
        const uint32_t cur_next = (b + 1 < bhi) ? band_cursors(b + 1) : 0u;   // prefetch
        // pack the entries reaching the band, clipped to it, in chunk order
        uint32_t n = 0;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t e0 = max(it.xs[j] & 0xFFFFu, bx0), e1 = min(it.xs[j] >> 16, bx1);
            const bool reach = e1 > e0;
            const uint64_t m = __ballot(reach);
            if (reach) {
                const uint32_t slot = n + lanes_below(m);
                s_g[slot] = it.g[j];
                s_x[slot] = (uint16_t)((e0 - bx0) | ((e1 - bx0) << 5));   // 0 <= e0 < e1 <= kBand
            }
            n += (uint32_t)__popcll(m);
        }
        __syncthreads();
        // column cursors increase along the row: the last one bounds them all
        const uint32_t cur_last = __builtin_amdgcn_readlane(cur_b, (int)(bx1 - bx0) - 1);
        if ((uint64_t)cur_last + n <= a.capacity)
            walk_band<false>(s_g, s_x, n, bx0, cur_b, a.values, a.capacity, lane);
        else
            walk_band<true>(s_g, s_x, n, bx0, cur_b, a.values, a.capacity, lane);
        __syncthreads();   // the LDS is free for the next band
        cur_b = cur_next;
    }
}

template <int kItems>
__global__ __launch_bounds__(64) void level2_scatter_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    __shared__ uint32_t s_g[kItems * 64];
    __shared__ uint16_t s_x[kItems * 64];
    const int lane = threadIdx.x;
    const int c2 = (int)a.info[kInfoC2];
    FOR_LEVEL2_CHUNK(c, c2) level2_scatter_chunk<kItems>(a, c, lane, s_g, s_x);
}

// Tile offsets from the scanned level-2 counts: tile (r, x) starts at chunk
// 0's cursor in column x of row r.  A row without chunks starts where the
// next row's block starts (the scan's running total there), or at the total
// K when it is the last.
__global__ __launch_bounds__(256) void tile_offsets_kernel(BinArgs a)
{
    if (a.skip && *a.skip) return;   // the last render's lists hold
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.tiles) return;
    const ViewParams& vp = a.views[view_of_tile(a.views, a.n_views, (uint32_t)t)];
    const int lt = (int)(t - vp.tile_base);
    const int r = (int)vp.row_base + lt / vp.tiles_x, x = lt % vp.tiles_x;
    const uint32_t* base = row_chunk_prefix(a);
    const uint32_t nch = base[r + 1] - base[r];
    const int64_t start = row_elem_prefix(a)[r];
    uint32_t off;
    if (nch > 0) off = a.counts2[start + (int64_t)x * nch];
    else if (start < (int64_t)a.info[kInfoC2Elems]) off = a.counts2[start];
    else off = a.tile_offsets[a.tiles];
    a.tile_offsets[t] = off;
}

unsigned grid8(int g) { return (unsigned)(8 * ((g + 7) / 8)); }
// level-2 waves launched at most (more chunks are taken in grid-stride turns)
constexpr int kMaxGrid2 = 65536;

}  // namespace

size_t bin_info_elems(int rows) { return (size_t)(kInfoRowChunks + 2 * (rows + 1) + 1); }
bool bin_items_supported(int items1, int items2)
{
    return (items1 == 4 || items1 == 8 || items1 == 16) && (items2 == 8 || items2 == 16 || items2 == 32);
}
bool tuning_supported(const Tuning& t)
{
    return depth_sort_items_supported(t.sort_items) && bin_items_supported(t.bin1_items, t.bin2_items) &&
           t.blend_group >= -1 && t.blend_group <= 64 &&
           (t.blend_batch == 128 || t.blend_batch == 256 || t.blend_batch == 512);
}
int bin_level1_chunks(int64_t n, int items1) { return (int)((n + (int64_t)items1 * 64 - 1) / ((int64_t)items1 * 64)); }
int bin_level2_chunk_bound(uint64_t row_entries, int rows, int items2)
{
    return (int)std::min<uint64_t>(row_entries / ((uint64_t)items2 * 64) + (uint64_t)rows + 1, 1u << 30);
}

namespace {
template <typename F>
void with_items1(int items, F f)
{
    switch (items) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 16>{}); break;
    }
}
template <typename F>
void with_items2(int items, F f)
{
    switch (items) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 32>{}); break;
    }
}
}  // namespace

// Level 1 up to the row offsets (R = rows_off[rows]) and the level-2 chunk
// table; no host dependence.
hipError_t launch_bin_rows(const BinArgs& a, uint64_t* scan_scratch, hipStream_t s)
{
    if (a.n == 0) {
        hipError_t e = launch_fill_u32(a.rows_off, 0u, a.rows + 1, s);
        if (e != hipSuccess) return e;
        return launch_fill_u32(a.info, 0u, (int64_t)bin_info_elems(a.rows), s);
    }
    if (!bin_items_supported(a.items1, a.items2)) return hipErrorInvalidValue;
    const int grid1 = a.chunks1 * a.n_views;
    with_items1(a.items1, [&](auto I) {
        hipLaunchKernelGGL(level1_count_kernel<decltype(I)::value>, dim3(grid8(grid1)), dim3(64),
                           (a.max_tiles_y + 1) * kDiffCopies * sizeof(uint32_t), s, a);
    });
    hipError_t e = launch_scan_exclusive(a.counts1, (int64_t)a.rows * a.chunks1, scan_scratch, nullptr,
                                         a.rows_off + a.rows, a.overflow, s, nullptr, a.skip);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(level2_table_kernel, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_row_scatter(const BinArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    if (!bin_items_supported(a.items1, a.items2)) return hipErrorInvalidValue;
    with_items1(a.items1, [&](auto I) {
        hipLaunchKernelGGL(level1_scatter_kernel<decltype(I)::value>, dim3(grid8(a.chunks1 * a.n_views)), dim3(64), 0,
                           s, a);
    });
    return hipGetLastError();
}

hipError_t launch_bin_tiles(const BinArgs& a, int grid2, uint64_t* scan_scratch, hipStream_t s)
{
    if (a.n == 0) return launch_fill_u32(a.tile_offsets, 0u, a.tiles + 1, s);
    if (!bin_items_supported(a.items1, a.items2)) return hipErrorInvalidValue;
    if (grid2 > 0)
        with_items2(a.items2, [&](auto I) {
            hipLaunchKernelGGL(level2_count_kernel<decltype(I)::value>, dim3(grid8(std::min(grid2, kMaxGrid2))),
                               dim3(64), (a.max_tiles_x + 1) * kDiffCopies * sizeof(uint32_t), s, a);
        });
    // the scan's length E2 is read on the device (info[1])
    hipError_t e = launch_scan_exclusive(a.counts2, (int64_t)a.counts2_capacity, scan_scratch, nullptr,
                                         a.tile_offsets + a.tiles, a.overflow, s, a.info + kInfoC2Elems, a.skip);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_offsets_kernel, dim3((unsigned)((a.tiles + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_tile_scatter(const BinArgs& a, int grid2, hipStream_t s)
{
    if (a.n == 0 || grid2 <= 0) return hipSuccess;
    if (!bin_items_supported(a.items1, a.items2)) return hipErrorInvalidValue;
    with_items2(a.items2, [&](auto I) {
        hipLaunchKernelGGL(level2_scatter_kernel<decltype(I)::value>, dim3(grid8(std::min(grid2, kMaxGrid2))),
                           dim3(64), 0, s, a);
    });
    return hipGetLastError();
}

}  // namespace gsmi
