// tile_bin.hip -- duplication of Gaussians into (tile, depth) pairs fused with
// the stable tile-digit pass of the key sort.
//
// Every Gaussian overlapping a screen tile (the 3-sigma square of Sec. 4.4)
// yields one pair; a pair's key is (tile << 32 | depth bits), its value the
// Gaussian index.  Gaussians arrive here already in (depth, index) order
// (depth_sort.hip), so a stable counting sort on the tile digit leaves every
// tile's list in front-to-back order: the output IS the sorted pair list.
//
// Work decomposition.  Tile rows are grouped into bands of at most
// kMaxBandTiles tiles (one LDS counter per tile of a band).  Per band, the
// pairs form one flat sequence in (depth order, tile row, tile column) order;
// its prefix over the depth-sorted Gaussians is one device-wide scan.  A
// wavefront owns a chunk of kChunkPairs consecutive pairs of one band, so
// every wave does the same amount of work however the pairs are spread over
// Gaussians (the big background Gaussians all sort to the back).
//   prep:    per sorted position, the pair count in each band
//   scan:    exclusive prefix of those counts (all bands in one sequence)
//   info:    band bases and chunk bases
//   count:   per chunk, an LDS histogram over the band's tiles
//   colscan: per tile, exclusive prefix over the band's chunks
//   offsets: exclusive scan of the tile totals -> tile_offsets
//   scatter: per chunk, LDS cursors at tile offset + chunk prefix; equal tiles
//            inside a 64-pair group are ranked by lane (ballot match), which
//            keeps depth order within every tile
#include "gs_internal.h"

namespace gsmi {
namespace {

__global__ __launch_bounds__(256) void band_prep_kernel(BinArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n) return;
    const int64_t nv = (int64_t)*a.n_visible;
    ushort4 r = make_ushort4(0, 0, 0, 0);
    if (k < nv) r = a.rect[a.sorted_idx[k]];
    a.rect_s[k] = r;
    const int w = (int)r.z - (int)r.x;
    for (int b = 0; b < a.num_bands; ++b) {
        const int b0 = b * a.band_rows, b1 = b0 + a.band_rows;
        const int y0 = (int)r.y > b0 ? (int)r.y : b0;
        const int y1 = (int)r.w < b1 ? (int)r.w : b1;
        a.bp[(int64_t)b * a.n + k] = (k < nv && y1 > y0) ? (uint32_t)(w * (y1 - y0)) : 0u;
    }
}

// band_info[0..B]: pair prefix at each band start (band_info[B] = K);
// band_info[B+1 .. 2B+1]: chunk prefix (band_info[2B+1] = number of chunks).
// With K >= 2^32 the 32-bit prefixes wrap: no chunk is handed out then (the
// overflow flag is already set by the scan).
__global__ void band_info_kernel(BinArgs a, const uint32_t* total32, const uint64_t* total64)
{
    if (threadIdx.x != 0) return;
    const int B = a.num_bands;
    const bool wrapped = *total64 > 0xFFFFFFFFull;
    uint32_t chunks = 0;
    for (int b = 0; b <= B; ++b) a.band_info[b] = (b < B) ? a.bp[(int64_t)b * a.n] : *total32;
    for (int b = 0; b < B; ++b) {
        a.band_info[B + 1 + b] = chunks;
        const uint32_t kb = a.band_info[b + 1] - a.band_info[b];
        if (!wrapped) chunks += (kb + kChunkPairs - 1) / kChunkPairs;
    }
    a.band_info[2 * B + 1] = chunks;
    if ((int64_t)chunks > (int64_t)a.max_chunks) {
        *a.overflow = 1u;
        a.band_info[2 * B + 1] = 0u;   // nothing is binned past the grid's room
    }
}

struct ChunkView {
    int band;
    uint32_t lo, hi;   // band-local pair range of the chunk
    uint32_t base;     // global prefix at the band start
    uint32_t kb;       // pairs in the band
    int64_t k0;        // last sorted position whose band prefix is <= lo
};

// Chunk of the workgroup: the dispatcher deals workgroups round-robin to the
// 8 XCDs, so block b takes chunk (b % 8) * ceil(grid / 8) + b / 8 and every
// XCD works through a contiguous run of chunks.  Consecutive chunks write
// adjacent pieces of each tile's list, which then meet in the same L2.
__device__ __forceinline__ int chunk_of_block()
{
    const int per_xcd = (int)((gridDim.x + 7) / 8);
    return (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
}

// Locates wave w's band and pair range, then k0 by a 64-ary search (each
// step probes 64 positions with one ballot).
__device__ __forceinline__ bool locate_chunk(const BinArgs& a, int w, int lane, ChunkView& v)
{
    const int B = a.num_bands;
    const uint32_t* info = a.band_info;
    if ((uint32_t)w >= info[2 * B + 1]) return false;
    int b = 0;
    while (b + 1 < B && info[B + 1 + b + 1] <= (uint32_t)w) ++b;
    const uint32_t c = (uint32_t)w - info[B + 1 + b];
    v.band = b;
    v.base = info[b];
    v.kb = info[b + 1] - info[b];
    v.lo = c * (uint32_t)kChunkPairs;
    v.hi = (v.lo + kChunkPairs < v.kb) ? v.lo + kChunkPairs : v.kb;
    const int64_t nv = (int64_t)*a.n_visible;
    const uint32_t* pre = a.bp + (int64_t)b * a.n;
    int64_t L = 0, R = nv;   // invariant: pre[L] - base <= lo
    while (R - L > 1) {
        const int64_t step = (R - L + 63) / 64;
        const int64_t q = L + (int64_t)lane * step;
        const bool ok = q < R && (pre[q] - v.base) <= v.lo;
        const uint64_t m = __ballot(ok);
        const int top = 63 - (int)__clzll((long long)m);
        const int64_t nl = L + (int64_t)top * step;
        R = (nl + step < R) ? nl + step : R;
        L = nl;
    }
    v.k0 = L;
    return true;
}

// Walks the pairs of one chunk 64 at a time; emit(local_tile, gaussian,
// active) is called by every lane of the wave for each group of 64 pairs.
template <class Emit>
__device__ __forceinline__ void walk_chunk(const BinArgs& a, const ChunkView& v, int lane, Emit&& emit)
{
    __shared__ uint32_t s_pre[64];
    __shared__ uint32_t s_x0w[64];   // x0 | w << 16
    __shared__ int s_row0[64];
    __shared__ uint32_t s_g[64];
    const int64_t nv = (int64_t)*a.n_visible;
    const uint32_t* pre_arr = a.bp + (int64_t)v.band * a.n;
    const int by0 = v.band * a.band_rows;
    for (int64_t kpos = v.k0; kpos < nv; kpos += 64) {
        const int64_t k = kpos + lane;
        uint32_t pre = v.kb, x0w = 1u << 16, g = 0;
        int row0 = 0;
        if (k < nv) {
            pre = pre_arr[k] - v.base;
            const ushort4 r = a.rect_s[k];
            const int y0 = (int)r.y > by0 ? (int)r.y : by0;
            x0w = (uint32_t)r.x | ((uint32_t)(r.z - r.x) << 16);
            row0 = y0 - by0;
            g = a.sorted_idx[k];
        }
        s_pre[lane] = pre;
        s_x0w[lane] = x0w;
        s_row0[lane] = row0;
        s_g[lane] = g;
        __syncthreads();
        // this batch holds the band pairs [pre of lane 0, pre of the next batch)
        const int64_t knext = kpos + 64;
        const uint32_t batch_end = (knext < nv) ? pre_arr[knext] - v.base : v.kb;
        const uint32_t p_start = (s_pre[0] > v.lo) ? s_pre[0] : v.lo;
        const uint32_t p_end = (batch_end < v.hi) ? batch_end : v.hi;
        for (uint32_t p0 = p_start; p0 < p_end; p0 += 64) {
            const uint32_t p = p0 + lane;
            const bool active = p < p_end;
            int local = 0;
            uint32_t gi = 0;
            if (active) {
                int lo = 0, hi = 63;   // last lane whose interval starts at or before p
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= p) lo = mid; else hi = mid - 1;
                }
                const uint32_t j = p - s_pre[lo];
                const uint32_t xw = s_x0w[lo];
                const int w = (int)(xw >> 16);
                // j / w for j, w <= 2^11: float estimate, then exact correction
                int row = (int)((float)j * __builtin_amdgcn_rcpf((float)w));
                int col = (int)j - row * w;
                if (col < 0) {
                    --row;
                    col += w;
                }
                if (col >= w) {
                    ++row;
                    col -= w;
                }
                local = (s_row0[lo] + row) * a.tiles_x + (int)(xw & 0xFFFFu) + col;
                gi = s_g[lo];
            }
            emit(local, gi, active);
        }
        __syncthreads();
        if (batch_end >= v.hi) break;
    }
}

__global__ __launch_bounds__(64) void bin_count_kernel(BinArgs a)
{
    __shared__ uint32_t cnt[kMaxBandTiles];
    const int lane = threadIdx.x;
    const int chunk = chunk_of_block();
    ChunkView v;
    if (!locate_chunk(a, chunk, lane, v)) return;
    const int by0 = v.band * a.band_rows;
    const int by1 = (by0 + a.band_rows < a.tiles_y) ? by0 + a.band_rows : a.tiles_y;
    const int band_tiles = (by1 - by0) * a.tiles_x;
    for (int k = lane; k < band_tiles; k += 64) cnt[k] = 0;
    __syncthreads();
    walk_chunk(a, v, lane, [&](int local, uint32_t, bool active) {
        if (active) atomicAdd(&cnt[local], 1u);
    });
    __syncthreads();
    uint32_t* dst = a.counts + (int64_t)chunk * kMaxBandTiles;
    for (int k = lane; k < band_tiles; k += 64) dst[k] = cnt[k];
}

// counts[chunk][t] -> exclusive prefix over the band's chunks (in place);
// tile totals -> tile_offsets[tile].  Block = (band, 64 tiles) x 16 segments.
__global__ __launch_bounds__(1024) void bin_colscan_kernel(BinArgs a)
{
    __shared__ uint32_t part[16][64];
    const int B = a.num_bands;
    const int groups = kMaxBandTiles / 64;
    const int band = blockIdx.x / groups, tg = blockIdx.x % groups;
    const int tl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int by0 = band * a.band_rows;
    const int by1 = (by0 + a.band_rows < a.tiles_y) ? by0 + a.band_rows : a.tiles_y;
    const int band_tiles = (by1 - by0) * a.tiles_x;
    const int t = tg * 64 + tl;
    const int c_begin = (int)a.band_info[B + 1 + band];
    const int c_end = (int)a.band_info[B + 1 + band + 1];
    const int per = (c_end - c_begin + 15) / 16;
    const int c0 = c_begin + seg * per;
    const int c1 = (c0 + per < c_end) ? c0 + per : c_end;
    const bool valid = t < band_tiles;
    uint32_t s = 0;
    if (valid)
        for (int c = c0; c < c1; ++c) s += a.counts[(int64_t)c * kMaxBandTiles + t];
    part[seg][tl] = s;
    __syncthreads();
    uint32_t run = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = part[k][tl];
        if (k < seg) run += x;
        tot += x;
    }
    if (valid) {
        for (int c = c0; c < c1; ++c) {
            const int64_t o = (int64_t)c * kMaxBandTiles + t;
            const uint32_t x = a.counts[o];
            a.counts[o] = run;
            run += x;
        }
        if (seg == 0) a.tile_offsets[(int64_t)by0 * a.tiles_x + t] = tot;
    }
}

__global__ __launch_bounds__(64) void bin_scatter_kernel(BinArgs a)
{
    __shared__ uint32_t cursor[kMaxBandTiles];
    const int lane = threadIdx.x;
    const int chunk = chunk_of_block();
    ChunkView v;
    if (!locate_chunk(a, chunk, lane, v)) return;
    const int by0 = v.band * a.band_rows;
    const int by1 = (by0 + a.band_rows < a.tiles_y) ? by0 + a.band_rows : a.tiles_y;
    const int band_tiles = (by1 - by0) * a.tiles_x;
    const uint32_t* prefix = a.counts + (int64_t)chunk * kMaxBandTiles;
    const uint32_t* toff = a.tile_offsets + (int64_t)by0 * a.tiles_x;
    for (int k = lane; k < band_tiles; k += 64) cursor[k] = toff[k] + prefix[k];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t cap = a.capacity;
    uint32_t* values = a.values;
    walk_chunk(a, v, lane, [&](int local, uint32_t g, bool active) {
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

hipError_t launch_bin_prepare(const BinArgs& a, uint64_t* scan_scratch, uint64_t* k_total, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(band_prep_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    // one exclusive scan over all bands' counts; its total is K
    uint32_t* total32 = a.band_info + 2 * a.num_bands + 2;   // slot after the table
    hipError_t e = launch_scan_exclusive(a.bp, (int64_t)a.num_bands * a.n, scan_scratch, k_total, total32,
                                         a.overflow, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(band_info_kernel, dim3(1), dim3(64), 0, s, a, (const uint32_t*)total32,
                       (const uint64_t*)k_total);
    return hipGetLastError();
}

hipError_t launch_bin_count(const BinArgs& a, int grid, hipStream_t s)
{
    if (a.n == 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)(8 * ((grid + 7) / 8))), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_offsets(const BinArgs& a, uint64_t* scan_scratch, hipStream_t s)
{
    const int64_t T = (int64_t)a.tiles_x * a.tiles_y;
    if (a.n == 0) return launch_fill_u32(a.tile_offsets, 0u, T + 1, s);
    hipLaunchKernelGGL(bin_colscan_kernel, dim3(a.num_bands * (kMaxBandTiles / 64)), dim3(1024), 0, s, a);
    return launch_scan_exclusive(a.tile_offsets, T, scan_scratch, nullptr, a.tile_offsets + T, nullptr, s);
}

hipError_t launch_bin_scatter(const BinArgs& a, int grid, hipStream_t s)
{
    if (a.n == 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3((unsigned)(8 * ((grid + 7) / 8))), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsmi
