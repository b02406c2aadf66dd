// gs_internal.h -- shared declarations of the gfx950 render kernels (not part
// of the public C ABI; see include/gsmi.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gsmi {

constexpr int kTile = 16;                 // screen tile edge in pixels
constexpr int kTilePixels = kTile * kTile;
constexpr int kMaxBandTiles = 2048;       // tile columns per image (width <= 32768)
constexpr int kSortBlock = 256;           // threads of a depth-sort block
constexpr int kTileWorkFields = 6;        // u64 fields of a per-tile blend trace record

// Launch shapes that change speed but never results (every choice gives the
// same image, lists and counts): chosen per workload by the autotuner.
struct Tuning {
    int sort_items;    // keys per thread of a depth-sort block: 4, 8, 16
    int bin1_items;    // depth-sorted Gaussians per lane of a level-1 binning wave: 4, 8, 16
    int bin2_items;    // row entries per lane of a level-2 binning wave: 8, 16, 32
    int blend_group;   // consecutive tiles dealt to one XCD by the blend: 1 .. 64;
                       // 0: tiles dispatched heaviest first, by the previous frame's work;
                       // -1: the same order as a work queue that a persistent grid drains
    int blend_batch;   // list entries the blend stages per batch: 128, 256, 512
};
constexpr Tuning kDefaultTuning = {8, 8, 16, 0, 256};
bool tuning_supported(const Tuning& t);
constexpr int kMaxRows = 2048;            // tile rows per image (height <= 32768)
constexpr int kMaxTotalRows = 16384;      // tile rows over all views of one render

// One projected Gaussian as the blend reads it: 3 x float4 = 48 bytes.
//   a = (u_hi, v_hi, u_lo, v_lo)   2D centre as a float pair of the double
//   b = (A, B, C, opacity)         conic and sigmoid(opacity logit)
//   c = (r, g, b, depth)
struct Splat {
    float4 a, b, c;
};

// One view of a render (a camera and its image), as the kernels read it from
// the device view table.  A single-image render is a table of one view.
struct ViewParams {
    double R[9], t[3];              // world -> camera, row-major
    double fx, fy, cx, cy, near_plane;
    float campos[3];                // camera centre -R^T t
    int width, height, tiles_x, tiles_y;
    uint32_t tile_base;             // global index of the view's first tile
    uint32_t row_base;              // global index of the view's first tile row
    float* out_rgb;                 // [3][H][W]
    float* out_T;                   // [H][W] or null
    uint32_t* out_nc;               // [H][W] or null
    // backward only: dL/d(out_rgb) [3][H][W] and dL/d(out_T) [H][W] or null
    const float* grad_rgb;
    const float* grad_T;
};

// Per-view counters written on the device: [0] Gaussians on screen (at least
// one tile), [1] Gaussians with a finite depth key (they sort first in a
// view's depth order; those culled or off screen have an empty rectangle),
// [2..3] pairs K of the view (u64).
constexpr int kViewCounters = 4;

// Finds the view owning global tile t (views hold ascending tile bases).
__device__ __forceinline__ int view_of_tile(const ViewParams* views, int n_views, uint32_t t)
{
    int lo = 0, hi = n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (views[mid].tile_base <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct ProjectArgs {
    int64_t n;                // Gaussians (per view)
    int sh_degree;
    int dtype;                // 0 f32, 1 bf16, 2 f16 (all but means)
    const float* means;
    const void* log_scales;
    const void* quats;
    const void* logits;
    const void* sh;
    const ViewParams* views;  // device table
    int n_views;
    // outputs per item v * n + i (view v, Gaussian i)
    Splat* splats;
    uint32_t* depth_key;
    int32_t* radius;
    uint32_t* tiles_touched;
    ushort4* rect;
    uint32_t* view_counts;        // [n_views][kViewCounters]
    uint32_t* partials;           // [blocks][n_views][4] per-block counts: on screen, pairs, keyed
    // when order is not null, one extra workgroup of the launch writes the
    // blend's dispatch order of order_tiles tiles, heaviest first by
    // order_cost (the previous frame's walked entries)
    const uint32_t* order_cost;
    uint32_t* order;
    int64_t order_tiles;
    // when not null: before its own stores each item compares its depth key
    // and rectangle with the values the buffers hold (the last render's);
    // the number that differ is added to changed[0] (zero before the launch)
    // and any difference clears changed[1] (one before the launch: the skip
    // flag of the sort and the binning while the previous lists hold)
    uint32_t* changed;
};

size_t project_partials_elems(int64_t n, int n_views);
hipError_t launch_project(const ProjectArgs& a, hipStream_t s);

// A tile rectangle (x0, y0, x1, y1; exclusive ends) packed in one word,
// x0 | x1 << 8 | y0 << 16 | y1 << 24, for views at most kPackedRectTiles
// tiles wide and tall: the payload the depth sort carries to the binning.
constexpr int kPackedRectTiles = 255;
__device__ __forceinline__ uint32_t pack_rect(ushort4 r)
{
    return (uint32_t)r.x | ((uint32_t)r.z << 8) | ((uint32_t)r.y << 16) | ((uint32_t)r.w << 24);
}
__device__ __forceinline__ ushort4 unpack_rect(uint32_t p)
{
    return make_ushort4((unsigned short)(p & 255u), (unsigned short)((p >> 16) & 255u),
                        (unsigned short)((p >> 8) & 255u), (unsigned short)(p >> 24));
}

// Stable LSD radix sort of the 32-bit keys of n_views segments of n items
// each, four 8-bit passes, every segment sorted on its own (values start as
// the item index v * n + i).  The sorted values end in vals_b; the sorted
// keys are not written (nothing reads them).  With rect (else null) each
// item carries its packed rectangle (pack_rect of rect[item]) through the
// passes, which ends in pay_b in the sorted order.
bool depth_sort_items_supported(int items);
size_t depth_sort_hist_elems(int64_t n, int n_views);   // enough for every supported width
hipError_t launch_depth_sort(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a,
                             uint32_t* keys_b, uint32_t* vals_b, const ushort4* rect, uint32_t* pay_a, uint32_t* pay_b,
                             uint32_t* counts, int64_t n, int n_views, int items, const uint32_t* reuse_words,
                             hipStream_t s);
// Reuse of the previous frame's order (one view, n items): reads the previous
// order from vals_b and this frame's keys; leaves in vals_b this frame's
// order when it can reach it cheaply, and in words[kReuseWords]: [0] 1 when
// vals_b holds the sorted order (launch_depth_sort then skips its passes),
// [1] descents of the previous order under this frame's keys, [2] 1 when the
// local repair ran.
constexpr int kReuseWords = 3;
size_t order_reuse_words(int64_t n);   // words and the gather's per-block counts
hipError_t launch_order_reuse(const uint32_t* keys, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                              uint32_t* vals_b, int64_t n, uint32_t* words, hipStream_t s);
// After launch_depth_sort with reuse words and rect: when the reused order
// held (words[0] = 1, so the passes did not run) writes pay_b[j] =
// pack_rect(rect[vals_b[j]]), the rectangles the passes would have carried;
// otherwise the passes wrote them and nothing is done.
hipError_t launch_order_pack(const uint32_t* vals_b, const ushort4* rect, int64_t n, const uint32_t* words,
                             uint32_t* pay_b, hipStream_t s);

struct BinArgs {
    const uint32_t* sorted_idx;   // [n_views * n] items (v * n + i), each view's segment in (depth, index) order
    const uint32_t* view_counts;  // device [n_views][kViewCounters]; keyed items sort first in a segment
    const ushort4* rect;          // [n_views * n] tile rectangle of each item in its view
    // the rectangles in depth order: packed (pack_rect), carried by the
    // depth sort, when sorted_pack is not null; else gathered from rect by
    // the row count into sorted_rect
    const uint32_t* sorted_pack;  // [n_views * n] or null
    ushort4* sorted_rect;         // [n_views * n] (keyed items; written by the row count)
    int64_t n;                    // Gaussians per view
    int n_views;
    const ViewParams* views;      // device table
    const uint32_t* row_tiles_x;  // [rows] tiles_x of each global tile row
    int rows;                     // global tile rows (sum of the views' tiles_y)
    int max_tiles_x, max_tiles_y; // largest tiles_x and tiles_y of the views
    int64_t tiles;                // global tiles (sum of the views' tiles)
    int items1, items2;           // items per lane of a level-1 / level-2 wave (Tuning)
    int chunks1;                  // level-1 chunks per view, bin_level1_chunks(n, items1)
    uint32_t* info;               // level-2 chunk table (bin_info_elems(rows))
    uint32_t* counts1;            // [rows][chunks1] counts -> exclusive scan = cursors
    uint32_t* rows_off;           // [rows + 1] row-list offsets; [rows] = R
    uint2* row_ent;               // [row_capacity] (item, x0 | x1 << 16)
    uint64_t row_capacity;
    uint32_t* counts2;            // per row: [tiles_x][row's chunks] counts -> scan = cursors
    uint64_t counts2_capacity;    // elements of counts2
    uint32_t* tile_offsets;       // [tiles + 1]; [tiles] = K
    uint32_t* values;             // [capacity] sorted pair values (items)
    uint64_t capacity;
    int max_chunks2;
    uint32_t* overflow;           // set to 1 when a capacity is exceeded
    // when not null, every binning kernel (and scan) reads *skip on the
    // device and does nothing when it is set: the lists, offsets and sizes of
    // the last render stay, because they are this render's
    const uint32_t* skip;
};

size_t bin_info_elems(int rows);
bool bin_items_supported(int items1, int items2);
int bin_level1_chunks(int64_t n, int items1);
int bin_level2_chunk_bound(uint64_t row_entries, int rows, int items2);
hipError_t launch_bin_rows(const BinArgs& a, uint64_t* scan_scratch, hipStream_t s);
hipError_t launch_bin_row_scatter(const BinArgs& a, hipStream_t s);
hipError_t launch_bin_tiles(const BinArgs& a, int grid2, uint64_t* scan_scratch, hipStream_t s);
hipError_t launch_bin_tile_scatter(const BinArgs& a, int grid2, hipStream_t s);
// info[] words the host reads after launch_bin_rows: level-2 chunks, level-2
// count elements
constexpr int kInfoC2 = 0;
constexpr int kInfoC2Elems = 1;

// Device-wide exclusive scan of n uint32 values in place; 64-bit total to
// *total64 and/or *total32 (either may be null), overflow flag when the total
// does not fit 32 bits.  block_scratch holds scan_scratch_elems(n) u64.
size_t scan_scratch_elems(int64_t n);
// With skip (else null) every kernel of the scan reads *skip on the device
// and does nothing when it is set.
hipError_t launch_scan_exclusive(uint32_t* data, int64_t n, uint64_t* block_scratch, uint64_t* total64,
                                 uint32_t* total32, uint32_t* overflow, hipStream_t s,
                                 const uint32_t* n_dev = nullptr, const uint32_t* skip = nullptr);

struct BlendArgs {
    const Splat* splats;
    const uint32_t* values;
    const uint32_t* tile_offsets;
    const ViewParams* views;   // device table: sizes, tile bases, outputs
    int n_views;
    int64_t tiles;             // global tiles
    int group;                 // tiles per XCD group (Tuning::blend_group)
    int batch;                 // list entries staged per batch (Tuning::blend_batch)
    const uint32_t* order;     // [tiles] dispatch order (block b renders order[b]), or null: XCD groups
    uint32_t* queue;           // with order: head of the work queue over order (zero before the launch),
                               // drained by a persistent grid; else null
    uint32_t* tile_cost;       // [tiles] list entries each tile walked before it finished, or null
    float bg[3];
    // per-tile trace when tracing (else null), [T][kTileWorkFields]: start
    // and end of the tile's workgroup (s_memrealtime, 100 MHz), entries
    // staged, wave bodies, (pixel, entry) evaluations up to each pixel's
    // termination, evaluations composited
    unsigned long long* tile_work;
};

hipError_t launch_blend(const BlendArgs& a, uint64_t capacity, hipStream_t s);

// Dispatch order of the blend: all tiles, heaviest first by cost[t] (the
// previous frame's walked entries), or by list length when cost is null;
// tiles of (nearly) equal cost in any order.  One workgroup.
hipError_t launch_blend_order(const uint32_t* cost, const uint32_t* tile_offsets, int64_t tiles, uint32_t* order,
                              hipStream_t s);

// Backward of the blend: per list entry, dL/d(u, v, A, B, C, opacity, r, g, b)
// summed over the pixels of every tile into grad2d[item][kGrad2d] (zeroed by
// the caller).  Reads each view's forward outputs and dL/d(out_rgb, out_T)
// from the view table.
constexpr int kGrad2d = 9;
struct BlendBackArgs {
    const Splat* splats;
    const uint32_t* values;
    const uint32_t* tile_offsets;
    const ViewParams* views;
    int n_views;
    int64_t tiles;
    int group;
    const uint32_t* order;   // the forward's dispatch order, or null: XCD groups
    float bg[3];
    float* grad2d;
};
hipError_t launch_blend_backward(const BlendBackArgs& a, uint64_t capacity, hipStream_t s);

// Backward of the projection: from grad2d of every (view, Gaussian) item to
// the gradients of the Gaussian parameters (float32, the input layouts),
// summed over the views.
struct ProjectBackArgs {
    int64_t n;
    int sh_degree;
    int dtype;
    const float* means;
    const void* log_scales;
    const void* quats;
    const void* logits;
    const void* sh;
    const ViewParams* views;
    int n_views;
    const float* grad2d;            // [n_views * n][kGrad2d]
    const uint32_t* tiles_touched;  // [n_views * n]: 0 for an item culled in its view
    float* g_means;                 // [3][n]
    float* g_log_scales;            // [3][n]
    float* g_quats;                 // [4][n]
    float* g_logits;                // [n]
    float* g_sh;                    // [(deg+1)^2][3][n]
};
hipError_t launch_project_backward(const ProjectBackArgs& a, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_write_keys(const uint32_t* values, const uint32_t* tile_offsets,
                             const uint32_t* depth_key, int64_t tiles, uint64_t* keys, hipStream_t s);

}  // namespace gsmi
