// api.hip -- host side of the C ABI declared in include/gsmi.h: argument
// validation, the context's device workspace and the launch sequence of one
// render of one or several views (project -> depth sort -> tile counts and
// offsets -> scatter -> blend).  A single-image render is the one-view case.
#include "gsmi.h"
#include "gs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace gsmi;

namespace {

thread_local std::string g_thread_error;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool fixed = false;   // a carve-out of the no-allocation scratch: never freed or grown
};

constexpr int kMaxViews = 1024;

// Workspace of gs_render_noalloc: every device buffer of such a render is
// carved out of this array, of which each device that loads the library
// holds one copy until the process ends.  Host code must never use the
// array's name as an address: the copy on device d lives at
// g_scratch_addr[d], taken once per device by gs_create.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mutex;
std::vector<void*> g_scratch_addr;   // per device: its copy of scratch, null until gs_create ran there

// With `device` current: records the address of that device's scratch.
hipError_t init_scratch_address(int device, int device_count)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if ((int)g_scratch_addr.size() < device_count) g_scratch_addr.resize((size_t)device_count, nullptr);
    if (g_scratch_addr[(size_t)device]) return hipSuccess;
    void* addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[(size_t)device] = addr;
    return hipSuccess;
}

void* scratch_address(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return (size_t)device < g_scratch_addr.size() ? g_scratch_addr[(size_t)device] : nullptr;
}

}  // namespace

// The device buffers of one render.  A context grows its own; a render of
// gs_render_noalloc carves fixed ones out of the static scratch array.
struct Workspace {
    DevBuf splats, depth_key, radius, tiles_touched, rect;
    DevBuf sort_ka, sort_va, sort_kb, sort_vb, hist, scan_scratch;
    DevBuf sort_pa, sort_pb;     // packed rectangles carried by the depth sort
    DevBuf bin_info, counts1, rows_off, row_ent, counts2, partials, sorted_rect, readback;
    DevBuf views, row_tiles_x;   // device view table and tiles_x of every global tile row
    DevBuf view_counts;          // [n_views][kViewCounters] visible Gaussians and pairs per view
    DevBuf counters;             // [1] capacity overflow flag
    DevBuf tile_offsets, values;
    DevBuf tile_work;   // per-tile blend trace [T][kTileWorkFields] u64 (GS_PROFILE_BLEND_WORK)
    DevBuf reuse_words;       // [kReuseWords] outcome of an order-reuse attempt
    // per-tile blend work of the last render, and the blend's dispatch order
    DevBuf tile_cost, tile_order;
};

struct gs_context {
    int device = 0;
    std::string err;
    Workspace ws;                    // buffers of the renders on this context
    uint32_t* host_info = nullptr;   // pinned readback of the per-frame sizes
    uint32_t* host_info_dev = nullptr;   // its device address: the size kernel writes there directly
    uint32_t profiling = 0;   // GS_PROFILE_* flags
    bool timed = false;       // the last render recorded stage events
    bool traced = false;      // the last render counted blend work
    // stage boundaries: 0 start, 1 project, 2 depth sort, 3 row counts,
    // 4 after the host read of K, 5 row scatter, 6 tile counts, 7 tile
    // scatter, 8 blend
    hipEvent_t ev[9] = {};
    // last render
    bool have_render = false;
    int64_t n = 0;
    int n_views = 0;
    int tiles_x = 0, tiles_y = 0;   // of the first view
    int64_t tiles = 0;              // global tiles over all views
    int rows = 0;                   // global tile rows
    uint64_t capacity = 0;
    int sorted_in_b = 1;
    hipStream_t stream = nullptr;
    hipEvent_t sizes_ev = nullptr;   // the host read of an eager render's sizes
    gs_graph* graph = nullptr;   // a captured render owns the workspace
    std::vector<ViewParams> last_views;   // view table of the last render
    gs_gaussians last_g{};                // scene of the last render
    float last_bg[3] = {0.f, 0.f, 0.f};
    DevBuf grad2d;                        // backward: per-item blend gradients
    DevBuf back_views;                    // backward: its own view table (a captured graph reads `views`)
    Tuning tuning = kDefaultTuning;       // launch shapes of the next render
    Tuning last_tuning = kDefaultTuning;  // launch shapes of the last render
    int64_t order_n = -1;     // items of the depth order the sort buffers hold (one view), -1 if none
    bool last_reuse = false;  // the last render started from the previous order
    // the tile lists in the workspace: those of a render of lists_n Gaussians
    // in views of the sizes lists_sizes (width, height per view) with pair
    // capacity lists_cap (0: eager)
    int64_t lists_n = -1;
    std::vector<int> lists_sizes;
    uint64_t lists_cap = 0;
    bool lists_compared = false;   // the last render compared keys and rectangles with its predecessor's
    std::vector<int> cost_layout;   // tiles_x, tiles_y of every view whose work ws.tile_cost holds
    // the last render was gs_render_noalloc: its sizes are in noalloc_info
    // (device words, allocated with the context), its buffers are gone
    bool last_noalloc = false;
    uint32_t* noalloc_info = nullptr;
};

struct gs_graph {
    gs_context* ctx = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<ViewParams> views;   // sizes and tile layout fixed at capture
};

namespace {

gs_status fail(gs_context* ctx, gs_status st, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    else g_thread_error = msg;
    return st;
}

gs_status hip_fail(gs_context* ctx, hipError_t e, const char* what)
{
    return fail(ctx, GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

gs_status ensure(gs_context* ctx, DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return GS_OK;
    if (b.fixed)
        return fail(ctx, GS_ERR_CAPACITY,
                    "a buffer of " + std::to_string(bytes) + " bytes does not fit its share of the no-allocation scratch");
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    const size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, GS_ERR_OUT_OF_MEMORY,
                    "hipMalloc of " + std::to_string(want) + " bytes failed: " + hipGetErrorString(e));
    }
    b.bytes = want;
    return GS_OK;
}

bool finite_all(const float* v, int k)
{
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

gs_status validate_gaussians(gs_context* ctx, const gs_gaussians* g)
{
    if (!g) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "gaussians is NULL");
    if (g->n < 0 || g->n >= (int64_t(1) << 31))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "n must lie in [0, 2^31)");
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "sh_degree must be 0..3");
    if (g->attr_dtype < GS_F32 || g->attr_dtype > GS_F16)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "attr_dtype must be GS_F32, GS_BF16 or GS_F16");
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "a Gaussian attribute pointer is NULL");
    return GS_OK;
}

gs_status validate_opts(gs_context* ctx, const gs_render_opts* opts)
{
    if (opts) {
        if (opts->tile_size != kTile) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "tile_size must be 16");
        if (opts->flags & ~(GS_RENDER_REUSE_ORDER | GS_RENDER_REUSE_LISTS))
            return fail(ctx, GS_ERR_INVALID_ARGUMENT, "unknown flag in opts->flags");
        if (opts->pair_capacity > 0xFFFFFFFFull)
            return fail(ctx, GS_ERR_UNSUPPORTED, "pair_capacity above 2^32-1: pair offsets are 32-bit");
        if (!finite_all(opts->background, 3))
            return fail(ctx, GS_ERR_INVALID_ARGUMENT, "background holds a non-finite value");
    }
    return GS_OK;
}

gs_status validate_view(gs_context* ctx, const gs_camera* cam, int32_t width, int32_t height, const float* out_rgb)
{
    if (!cam) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    if (!out_rgb) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "out_rgb is NULL");
    if (width < 1 || height < 1 || width > 32768 || height > 32768)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "width and height must lie in [1, 32768]");
    const int tiles_x = (width + kTile - 1) / kTile;
    if (tiles_x > kMaxBandTiles) return fail(ctx, GS_ERR_UNSUPPORTED, "image wider than 32768 pixels");
    if (!finite_all(cam->R, 9) || !finite_all(cam->t, 3) || !std::isfinite(cam->fx) || !std::isfinite(cam->fy) ||
        !std::isfinite(cam->cx) || !std::isfinite(cam->cy) || !std::isfinite(cam->near_plane))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "camera holds a non-finite value");
    if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !(cam->near_plane > 0.f))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "camera fx, fy and near_plane must be positive");
    return GS_OK;
}

gs_status validate(gs_context* ctx, const gs_gaussians* g, const gs_camera* cam, int32_t width, int32_t height,
                   const gs_render_opts* opts, const float* out_rgb)
{
    gs_status st = validate_gaussians(ctx, g);
    if (st == GS_OK) st = validate_view(ctx, cam, width, height, out_rgb);
    if (st == GS_OK) st = validate_opts(ctx, opts);
    return st;
}

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

// records the boundary event k when stage timing is on
#define STAGE_MARK(k)                                                               \
    do {                                                                            \
        if (ctx->profiling & GS_PROFILE_STAGES) HIP_TRY(hipEventRecord(ctx->ev[(k)], s), "hipEventRecord"); \
    } while (0)


// The view table is written by a kernel whose arguments carry up to
// kViewsPerLaunch views (kernel arguments are copied at launch, so the host
// array can be reused at once and the upload stays on the compute queue).
constexpr int kViewsPerLaunch = 16;
// counters[kCounterChanged]: the projection's count of (view, Gaussian)
// items whose depth key or rectangle differ from the last render's (list
// reuse), and after it the flag that none did: set to 1 at frame set-up when
// the comparison runs, cleared by any view that finds a change
constexpr int kCounterChanged = 2;
// counters[kCounterBlendQueue]: head of the blend's work queue (blend_group -1)
constexpr int kCounterBlendQueue = 4;

struct ViewBatch {
    ViewParams v[kViewsPerLaunch];
};
static_assert(sizeof(ViewBatch) <= 4000, "kernel argument size");

__global__ void write_views_kernel(ViewBatch b, int count, ViewParams* dst)
{
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&b.v[0]);
    uint32_t* out = reinterpret_cast<uint32_t*>(dst);
    const int words = count * (int)(sizeof(ViewParams) / 4);
    for (int k = threadIdx.x; k < words; k += blockDim.x) out[k] = src[k];
}

// The start of a frame of at most kViewsPerLaunch views in one launch: the
// overflow counters cleared, the view table written (when `write`) and the
// tiles_x of every global tile row, all from the views in the arguments.
__global__ void frame_setup_kernel(ViewBatch b, int count, ViewParams* dst, int write, uint32_t* counters,
                                   uint32_t* row_tiles_x, int rows, uint32_t hold_init)
{
    if (threadIdx.x < 16) counters[threadIdx.x] = threadIdx.x == kCounterChanged + 1 ? hold_init : 0u;
    if (write) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&b.v[0]);
        uint32_t* out = reinterpret_cast<uint32_t*>(dst);
        const int words = count * (int)(sizeof(ViewParams) / 4);
        for (int k = threadIdx.x; k < words; k += blockDim.x) out[k] = src[k];
    }
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        int v = 0;
        while (v + 1 < count && (int)b.v[v + 1].row_base <= r) ++v;
        row_tiles_x[r] = (uint32_t)b.v[v].tiles_x;
    }
}

hipError_t write_view_table(const std::vector<ViewParams>& hv, ViewParams* dst, hipStream_t s)
{
    for (size_t v0 = 0; v0 < hv.size(); v0 += kViewsPerLaunch) {
        ViewBatch b;
        const int cnt = (int)std::min<size_t>(kViewsPerLaunch, hv.size() - v0);
        std::memcpy(b.v, hv.data() + v0, (size_t)cnt * sizeof(ViewParams));
        hipLaunchKernelGGL(write_views_kernel, dim3(1), dim3(256), 0, s, b, cnt, dst + v0);
    }
    return hipGetLastError();
}

// tiles_x of every global tile row (rows of view v are [row_base, row_base + tiles_y))
// The eager render's host read gathered for one copy: the view counters
// ([n][kViewCounters]), then counters[0..3], R and the level-2 chunk and
// count-element totals.
constexpr int kReadbackTail = 7;
__global__ void pack_readback_kernel(const uint32_t* view_counts, int n_vc, const uint32_t* counters,
                                     const uint32_t* r_total, const uint32_t* info, uint32_t* out)
{
    for (int i = threadIdx.x; i < n_vc + kReadbackTail; i += blockDim.x) {
        const int t = i - n_vc;
        out[i] = i < n_vc ? view_counts[i] : (t < 4 ? counters[t] : (t == 4 ? *r_total : info[t - 5]));
    }
    __threadfence_system();   // out may be pinned host memory, read by the host after the frame's event
}

__global__ void row_table_kernel(const ViewParams* views, int n_views, uint32_t* row_tiles_x, int rows)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    int lo = 0, hi = n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)views[mid].row_base <= r) lo = mid;
        else hi = mid;
    }
    row_tiles_x[r] = (uint32_t)views[lo].tiles_x;
}


// One render of n_views views of the scene g (validated by the caller).
// write_table: upload the view table first (false while a graph is captured:
// the graph then reads the table its owner writes before each launch).
gs_status render_views(gs_context* ctx, const gs_gaussians* g, const std::vector<ViewParams>& hv,
                       const gs_render_opts* opts, hipStream_t s, bool write_table = true,
                       Workspace* fixed_ws = nullptr)
{
    gs_status st;
    gs_render_opts o{};
    o.tile_size = kTile;
    if (opts) o = *opts;
    // fixed_ws: the buffers of a no-allocation render (capacity mode, no
    // order reuse, no work tracing, no per-tile history: the scratch is
    // shared by every context on the device)
    Workspace& w = fixed_ws ? *fixed_ws : ctx->ws;
    const bool noalloc = fixed_ws != nullptr;
    if (noalloc && o.pair_capacity == 0) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "no-allocation render without a capacity");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    ctx->have_render = false;
    ctx->last_noalloc = false;
    const int64_t prev_order_n = ctx->order_n;
    ctx->order_n = -1;   // valid again only once this render has completed its sort
    const int64_t prev_lists_n = ctx->lists_n;
    ctx->lists_n = -1;   // valid again only once this render has completed its lists
    ctx->lists_compared = false;

    const int V = (int)hv.size();
    const int64_t n = g->n;
    const int64_t items = n * V;
    const int rows = (int)(hv.back().row_base + hv.back().tiles_y);
    const int64_t T = (int64_t)hv.back().tile_base + (int64_t)hv.back().tiles_x * hv.back().tiles_y;
    int max_tx = 0, max_ty = 0;
    for (const ViewParams& v : hv) {
        max_tx = std::max(max_tx, v.tiles_x);
        max_ty = std::max(max_ty, v.tiles_y);
    }
    const size_t ni = (size_t)(items > 0 ? items : 1);
    const Tuning tu = ctx->tuning;
    const int chunks1 = std::max(bin_level1_chunks(n, tu.bin1_items), 1);

    if ((st = ensure(ctx, w.splats, ni * sizeof(Splat))) != GS_OK) return st;
    if ((st = ensure(ctx, w.depth_key, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.radius, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.tiles_touched, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.rect, ni * 8)) != GS_OK) return st;
    if ((st = ensure(ctx, w.sorted_rect, ni * 8)) != GS_OK) return st;
    if ((st = ensure(ctx, w.sort_ka, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.sort_va, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.sort_kb, ni * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.sort_vb, ni * 4)) != GS_OK) return st;
    const bool fits_packed = !noalloc && max_tx <= kPackedRectTiles && max_ty <= kPackedRectTiles;
    if (fits_packed) {
        if ((st = ensure(ctx, w.sort_pa, ni * 4)) != GS_OK) return st;
        if ((st = ensure(ctx, w.sort_pb, ni * 4)) != GS_OK) return st;
    }
    if ((st = ensure(ctx, w.hist, depth_sort_hist_elems(n, V) * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.partials, project_partials_elems(n, V) * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.views, (size_t)V * sizeof(ViewParams))) != GS_OK) return st;
    if ((st = ensure(ctx, w.view_counts, (size_t)V * kViewCounters * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.row_tiles_x, (size_t)rows * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.bin_info, bin_info_elems(rows) * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.rows_off, (size_t)(rows + 1) * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.counts1, (size_t)chunks1 * rows * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.counters, 64)) != GS_OK) return st;
    if ((st = ensure(ctx, w.tile_offsets, (size_t)(T + 1) * 4)) != GS_OK) return st;
    // every blend records its tiles' work; with blend_group 0 it is dispatched
    // (with -1 queued for a persistent grid) heaviest first, by the last
    // render's work when that render had the same tile layout (the history:
    // ordered by one extra workgroup of the projection launch), else by list
    // length (ordered before the blend)
    std::vector<int> layout;
    for (const ViewParams& v : hv) {
        layout.push_back(v.tiles_x);
        layout.push_back(v.tiles_y);
    }
    const void* cost_before = w.tile_cost.p;
    if ((st = ensure(ctx, w.tile_cost, (size_t)std::max<int64_t>(T, 1) * 4)) != GS_OK) return st;
    const bool history = !noalloc && cost_before == w.tile_cost.p && ctx->cost_layout == layout;
    if (tu.blend_group <= 0)
        if ((st = ensure(ctx, w.tile_order, (size_t)std::max<int64_t>(T, 1) * 4)) != GS_OK) return st;
    const bool order_in_project = tu.blend_group <= 0 && history && n > 0;
    // list reuse: the workspace holds the lists of a render of as many
    // Gaussians in views of the same sizes, with the same pair capacity (a
    // capacity that truncated them truncates an identical frame's the same
    // way); the projection counts the items whose depth key or rectangle
    // changed since, and when none did those lists are this frame's (they
    // depend on nothing else): the sort and the binning then skip on the
    // device
    std::vector<int> sizes;
    for (const ViewParams& v : hv) {
        sizes.push_back(v.width);
        sizes.push_back(v.height);
    }
    const bool try_lists = !noalloc && (o.flags & GS_RENDER_REUSE_LISTS) && n > 0 && prev_lists_n == n &&
                           ctx->lists_sizes == sizes && ctx->lists_cap == o.pair_capacity;

    ViewParams* views = static_cast<ViewParams*>(w.views.p);
    uint32_t* counters = static_cast<uint32_t*>(w.counters.p);
    uint32_t* view_counts = static_cast<uint32_t*>(w.view_counts.p);
    if (V <= kViewsPerLaunch) {
        ViewBatch b;
        std::memcpy(b.v, hv.data(), (size_t)V * sizeof(ViewParams));
        hipLaunchKernelGGL(frame_setup_kernel, dim3(1), dim3(256), 0, s, b, V, views, write_table ? 1 : 0, counters,
                           static_cast<uint32_t*>(w.row_tiles_x.p), rows, try_lists ? 1u : 0u);
    } else {
        HIP_TRY(launch_fill_u32(counters, 0u, 16, s), "clear counters");
        if (try_lists) HIP_TRY(launch_fill_u32(counters + kCounterChanged + 1, 1u, 1, s), "list reuse flag");
        if (write_table) HIP_TRY(write_view_table(hv, views, s), "view table");
        hipLaunchKernelGGL(row_table_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                           (const ViewParams*)views, V, static_cast<uint32_t*>(w.row_tiles_x.p), rows);
    }
    HIP_TRY(hipGetLastError(), "frame set-up");
    STAGE_MARK(0);

    // list reuse: the workspace holds the lists of a one-view render of as
    // many Gaussians at the same size and pair capacity (a capacity that
    // truncated them truncates an identical frame's the same way); the
    // projection counts the Gaussians whose depth key or rectangle changed
    // since, and when none did those lists are this frame's (they depend on
    // nothing else): the sort and the binning then skip on the device

    ProjectArgs pa{};
    pa.n = n;
    pa.sh_degree = g->sh_degree;
    pa.dtype = g->attr_dtype;
    pa.means = g->means;
    pa.log_scales = g->log_scales;
    pa.quats = g->quats;
    pa.logits = g->opacity_logits;
    pa.sh = g->sh;
    pa.views = views;
    pa.n_views = V;
    pa.splats = static_cast<Splat*>(w.splats.p);
    pa.depth_key = static_cast<uint32_t*>(w.depth_key.p);
    pa.radius = static_cast<int32_t*>(w.radius.p);
    pa.tiles_touched = static_cast<uint32_t*>(w.tiles_touched.p);
    pa.rect = static_cast<ushort4*>(w.rect.p);
    pa.view_counts = view_counts;
    pa.partials = static_cast<uint32_t*>(w.partials.p);
    if (order_in_project) {
        pa.order_cost = static_cast<const uint32_t*>(w.tile_cost.p);
        pa.order = static_cast<uint32_t*>(w.tile_order.p);
        pa.order_tiles = T;
    }
    // counters[kCounterChanged]: the changed count, then the flag that the
    // previous lists hold, which every kernel of the sort and the binning
    // reads on the device
    pa.changed = try_lists ? counters + kCounterChanged : nullptr;
    HIP_TRY(launch_project(pa, s), "project");
    STAGE_MARK(1);
    ctx->lists_compared = try_lists;

    BinArgs ba{};
    ba.view_counts = view_counts;
    ba.rect = pa.rect;
    ba.sorted_rect = static_cast<ushort4*>(w.sorted_rect.p);
    ba.n = n;
    ba.n_views = V;
    ba.views = views;
    ba.row_tiles_x = static_cast<const uint32_t*>(w.row_tiles_x.p);
    ba.rows = rows;
    ba.max_tiles_x = max_tx;
    ba.max_tiles_y = max_ty;
    ba.tiles = T;
    ba.items1 = tu.bin1_items;
    ba.items2 = tu.bin2_items;
    ba.chunks1 = chunks1;
    ba.info = static_cast<uint32_t*>(w.bin_info.p);
    ba.counts1 = static_cast<uint32_t*>(w.counts1.p);
    ba.rows_off = static_cast<uint32_t*>(w.rows_off.p);
    ba.tile_offsets = static_cast<uint32_t*>(w.tile_offsets.p);
    ba.overflow = counters + 1;
    uint64_t capacity = o.pair_capacity;
    int in_b = 1;
    ba.skip = try_lists ? counters + kCounterChanged + 1 : nullptr;
    // pair_capacity > 0: every size below is the bound the capacity implies
    // (row entries <= pairs); else the host reads K, R and the level-2 sizes
    // once
    ba.row_capacity = capacity ? capacity : ~0ull;
    ba.max_chunks2 = capacity ? bin_level2_chunk_bound(capacity, rows, tu.bin2_items) : (1 << 30);
    ba.counts2_capacity = capacity ? (uint64_t)ba.max_chunks2 * max_tx : ~0ull;
    // scan lengths: level-1 counts, tile offsets and
    // (pair_capacity > 0) the level-2 counts; the eager path grows the scratch
    // for the level-2 counts after its host read
    int64_t scan_max = std::max<int64_t>(T + 1, (int64_t)rows * chunks1);
    if (capacity) scan_max = std::max<int64_t>(scan_max, (int64_t)ba.counts2_capacity);
    if ((st = ensure(ctx, w.scan_scratch, scan_scratch_elems(scan_max) * 8)) != GS_OK) return st;
    uint64_t* scan_scratch = static_cast<uint64_t*>(w.scan_scratch.p);
    // one view of the same Gaussians as the last render: start from its order
    const bool reuse = !noalloc && (o.flags & GS_RENDER_REUSE_ORDER) && V == 1 && n > 0 && prev_order_n == n;
    uint32_t* reuse_words = nullptr;
    if (reuse) {
        if ((st = ensure(ctx, w.reuse_words, order_reuse_words(n) * 4)) != GS_OK) return st;
        reuse_words = static_cast<uint32_t*>(w.reuse_words.p);
        HIP_TRY(launch_order_reuse(pa.depth_key, static_cast<uint32_t*>(w.sort_ka.p),
                                   static_cast<uint32_t*>(w.sort_va.p), static_cast<uint32_t*>(w.sort_kb.p),
                                   static_cast<uint32_t*>(w.sort_vb.p), n, reuse_words, s),
                "order reuse");
    }
    // the sort carries each Gaussian's packed rectangle to the binning, which
    // then reads the rectangles in depth order instead of gathering them (not
    // in a no-allocation render: its scratch is kept small); when a reused
    // order skips the radix passes, one gather in that order writes them
    const bool packed = fits_packed;
    HIP_TRY(launch_depth_sort(pa.depth_key, static_cast<uint32_t*>(w.sort_ka.p),
                              static_cast<uint32_t*>(w.sort_va.p), static_cast<uint32_t*>(w.sort_kb.p),
                              static_cast<uint32_t*>(w.sort_vb.p), packed ? pa.rect : nullptr,
                              static_cast<uint32_t*>(packed ? w.sort_pa.p : nullptr),
                              static_cast<uint32_t*>(packed ? w.sort_pb.p : nullptr),
                              static_cast<uint32_t*>(w.hist.p),
                              n, V, tu.sort_items, reuse ? reuse_words : ba.skip, s),
            "depth sort");
    if (reuse && packed)
        HIP_TRY(launch_order_pack(static_cast<const uint32_t*>(w.sort_vb.p), pa.rect, n, reuse_words,
                                  static_cast<uint32_t*>(w.sort_pb.p), s),
                "reused order's rectangles");
    ba.sorted_idx = static_cast<const uint32_t*>(w.sort_vb.p);
    ba.sorted_pack = packed ? static_cast<const uint32_t*>(w.sort_pb.p) : nullptr;
    STAGE_MARK(2);
    HIP_TRY(launch_bin_rows(ba, scan_scratch, s), "bin rows");
    STAGE_MARK(3);

    int grid2 = ba.max_chunks2;
    bool rows_scattered = false;   // the row scatter ran while the host read the sizes
    bool lists_held = false;       // the host read that the previous lists hold (eager)
    if (capacity == 0) {
        // eager: one host read (one copy) of the per-view pairs, R and the
        // level-2 sizes
        uint32_t* hi = ctx->host_info;
        const int n_vc = V * kViewCounters;
        // the sizes go straight into the pinned host buffer (its device
        // address), else through a device buffer and a copy; the event below
        // marks their arrival
        uint32_t* rb = ctx->host_info_dev;
        if (!rb) {
            if ((st = ensure(ctx, w.readback, (size_t)(n_vc + kReadbackTail) * 4)) != GS_OK) return st;
            rb = static_cast<uint32_t*>(w.readback.p);
        }
        hipLaunchKernelGGL(pack_readback_kernel, dim3(1), dim3(256), 0, s, (const uint32_t*)view_counts, n_vc,
                           (const uint32_t*)counters, (const uint32_t*)(ba.rows_off + rows),
                           (const uint32_t*)ba.info,
                           rb);
        HIP_TRY(hipGetLastError(), "read sizes");
        if (!ctx->host_info_dev)
            HIP_TRY(hipMemcpyAsync(hi, rb, (size_t)(n_vc + kReadbackTail) * 4, hipMemcpyDeviceToHost, s),
                    "read sizes");
        // the row scatter needs no size but R, and the row-entry buffer of
        // earlier renders mostly holds this frame's entries: it runs while
        // the host reads the sizes, and runs again into a grown buffer when R
        // exceeds it (its stores past the buffer are dropped)
        const uint64_t spec = w.row_ent.bytes / 8;
        if (spec > 0) {
            HIP_TRY(hipEventRecord(ctx->sizes_ev, s), "hipEventRecord");
            ba.row_ent = static_cast<uint2*>(w.row_ent.p);
            ba.row_capacity = spec;
            STAGE_MARK(4);
            HIP_TRY(launch_bin_row_scatter(ba, s), "bin row scatter");
            STAGE_MARK(5);
            rows_scattered = true;
            HIP_TRY(hipEventSynchronize(ctx->sizes_ev), "hipEventSynchronize");
        } else {
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        uint32_t* tail = hi + n_vc;
        uint64_t K64 = 0;
        for (int v = 0; v < V; ++v) {
            const uint32_t* c = hi + (size_t)v * kViewCounters;
            K64 += (uint64_t)c[2] | ((uint64_t)c[3] << 32);
        }
        if (K64 > 0xFFFFFFFFull || tail[1] != 0u)
            return fail(ctx, GS_ERR_CAPACITY, "more than 2^32-1 (Gaussian, tile) pairs");
        capacity = K64;
        ba.row_capacity = tail[4];
        if (rows_scattered && ba.row_capacity > spec) {
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");   // the buffer is grown below
            rows_scattered = false;
        }
        grid2 = (int)tail[5];
        ba.max_chunks2 = grid2;
        ba.counts2_capacity = tail[6];
        // counters[kCounterChanged + 1] came with the sizes: when the lists
        // hold, the tile-level launches (which would skip) are not made
        lists_held = try_lists && tail[kCounterChanged + 1] != 0u;
    }
    ba.capacity = capacity;
    // in eager mode nothing queued uses the buffers grown here (the kernels
    // before the host read have completed; a row scatter still running uses
    // the row-entry buffer, which then has room)
    if ((st = ensure(ctx, w.scan_scratch, scan_scratch_elems((int64_t)std::max<uint64_t>(ba.counts2_capacity, 1)) *
                                                 8)) != GS_OK)
        return st;
    scan_scratch = static_cast<uint64_t*>(w.scan_scratch.p);
    const size_t rows_cap = (size_t)std::max<uint64_t>(ba.row_capacity, 1);
    if ((st = ensure(ctx, w.row_ent, rows_cap * 8)) != GS_OK) return st;
    if ((st = ensure(ctx, w.counts2, (size_t)std::max<uint64_t>(ba.counts2_capacity, 1) * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, w.values, (size_t)std::max<uint64_t>(capacity, 1) * 4)) != GS_OK) return st;
    ba.row_ent = static_cast<uint2*>(w.row_ent.p);
    ba.counts2 = static_cast<uint32_t*>(w.counts2.p);
    ba.values = static_cast<uint32_t*>(w.values.p);
    if (!rows_scattered) {
        STAGE_MARK(4);
        HIP_TRY(launch_bin_row_scatter(ba, s), "bin row scatter");
        STAGE_MARK(5);
    }
    if (!lists_held) HIP_TRY(launch_bin_tiles(ba, grid2, scan_scratch, s), "bin tile counts");
    STAGE_MARK(6);
    if (!lists_held) HIP_TRY(launch_bin_tile_scatter(ba, grid2, s), "bin tile scatter");
    STAGE_MARK(7);

    BlendArgs bl{};
    bl.splats = pa.splats;
    bl.values = ba.values;
    bl.tile_offsets = ba.tile_offsets;
    bl.views = views;
    bl.n_views = V;
    bl.tiles = T;
    bl.group = tu.blend_group;
    bl.batch = tu.blend_batch;
    const float zero_bg[3] = {0.f, 0.f, 0.f};
    const float* bg = opts ? o.background : zero_bg;
    for (int k = 0; k < 3; ++k) bl.bg[k] = bg[k];
    bl.tile_work = nullptr;
    if ((ctx->profiling & GS_PROFILE_BLEND_WORK) && !noalloc) {
        if ((st = ensure(ctx, w.tile_work, (size_t)std::max<int64_t>(T, 1) * kTileWorkFields * 8)) != GS_OK)
            return st;
        bl.tile_work = static_cast<unsigned long long*>(w.tile_work.p);
    }
    bl.tile_cost = static_cast<uint32_t*>(w.tile_cost.p);
    bl.order = nullptr;
    bl.queue = nullptr;
    if (tu.blend_group <= 0) {
        uint32_t* order = static_cast<uint32_t*>(w.tile_order.p);
        // ordered by the projection's extra workgroup, or here by list length
        if (!order_in_project)
            HIP_TRY(launch_blend_order(nullptr, bl.tile_offsets, T, order, s), "blend order");
        bl.order = order;
        // the queue head was cleared with the frame's counters
        if (tu.blend_group < 0) bl.queue = counters + kCounterBlendQueue;
    }
    HIP_TRY(launch_blend(bl, capacity, s), "blend");
    STAGE_MARK(8);
    if (noalloc) {
        // nothing of this render stays with the context but its sizes: the
        // next render on the device may overwrite the scratch
        hipLaunchKernelGGL(pack_readback_kernel, dim3(1), dim3(256), 0, s, (const uint32_t*)view_counts,
                           kViewCounters, (const uint32_t*)counters, (const uint32_t*)(ba.rows_off + rows),
                           (const uint32_t*)ba.info, ctx->noalloc_info);
        HIP_TRY(hipGetLastError(), "pack sizes");
        ctx->last_noalloc = true;
        ctx->n = n;
        ctx->n_views = V;
        ctx->tiles_x = hv[0].tiles_x;
        ctx->tiles_y = hv[0].tiles_y;
        ctx->tiles = T;
        ctx->rows = rows;
        ctx->capacity = capacity;
        ctx->stream = s;
        ctx->cost_layout.clear();
        ctx->have_render = false;
        ctx->order_n = -1;
        ctx->timed = (ctx->profiling & GS_PROFILE_STAGES) != 0;
        ctx->traced = false;
        return GS_OK;
    }
    ctx->cost_layout = layout;

    ctx->have_render = true;
    ctx->last_tuning = tu;
    ctx->order_n = (V == 1 && in_b) ? n : -1;
    ctx->last_reuse = reuse;
    ctx->lists_n = n;
    ctx->lists_sizes = sizes;
    ctx->lists_cap = o.pair_capacity;
    ctx->last_views = hv;
    ctx->last_g = *g;
    for (int k = 0; k < 3; ++k) ctx->last_bg[k] = bl.bg[k];
    ctx->timed = (ctx->profiling & GS_PROFILE_STAGES) != 0;
    ctx->traced = bl.tile_work != nullptr;
    ctx->n = n;
    ctx->n_views = V;
    ctx->tiles_x = hv[0].tiles_x;
    ctx->tiles_y = hv[0].tiles_y;
    ctx->tiles = T;
    ctx->rows = rows;
    ctx->capacity = capacity;
    ctx->sorted_in_b = in_b;
    ctx->stream = s;
    return GS_OK;
}

gs_status build_views(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                      const gs_render_opts* opts, std::vector<ViewParams>& hv);

// Bytes of the buffers a capacity-mode render of the views hv asks for (the
// sizes render_views requests, each rounded up to 256 bytes).  With w, the
// buffers are also laid out one after another from base and marked fixed.
size_t carve_noalloc(Workspace* w, unsigned char* base, int64_t n, const std::vector<ViewParams>& hv, const Tuning& tu,
                     uint64_t capacity)
{
    Workspace dummy;
    Workspace& ws = w ? *w : dummy;
    size_t off = 0;
    auto take = [&](DevBuf& b, size_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (w) {
            b.p = base + off;
            b.bytes = bytes;
            b.fixed = true;
        }
        off += bytes;
    };
    const int V = (int)hv.size();
    const size_t ni = (size_t)std::max<int64_t>(n * V, 1);
    const int rows = (int)(hv.back().row_base + hv.back().tiles_y);
    const int64_t T = (int64_t)hv.back().tile_base + (int64_t)hv.back().tiles_x * hv.back().tiles_y;
    int max_tx = 0;
    for (const ViewParams& v : hv) max_tx = std::max(max_tx, v.tiles_x);
    const int chunks1 = std::max(bin_level1_chunks(n, tu.bin1_items), 1);
    const int max_chunks2 = bin_level2_chunk_bound(capacity, rows, tu.bin2_items);
    const uint64_t counts2_cap = (uint64_t)max_chunks2 * max_tx;
    const int64_t scan_max = std::max<int64_t>(std::max<int64_t>(T + 1, (int64_t)rows * chunks1), (int64_t)counts2_cap);
    take(ws.splats, ni * sizeof(Splat));
    take(ws.depth_key, ni * 4);
    take(ws.radius, ni * 4);
    take(ws.tiles_touched, ni * 4);
    take(ws.rect, ni * 8);
    take(ws.sorted_rect, ni * 8);
    take(ws.sort_ka, ni * 4);
    take(ws.sort_va, ni * 4);
    take(ws.sort_kb, ni * 4);
    take(ws.sort_vb, ni * 4);
    take(ws.hist, depth_sort_hist_elems(n, V) * 4);
    take(ws.partials, project_partials_elems(n, V) * 4);
    take(ws.views, (size_t)V * sizeof(ViewParams));
    take(ws.view_counts, (size_t)V * kViewCounters * 4);
    take(ws.row_tiles_x, (size_t)rows * 4);
    take(ws.bin_info, bin_info_elems(rows) * 4);
    take(ws.rows_off, (size_t)(rows + 1) * 4);
    take(ws.counts1, (size_t)chunks1 * rows * 4);
    take(ws.counters, 64);
    take(ws.tile_offsets, (size_t)(T + 1) * 4);
    take(ws.scan_scratch, scan_scratch_elems(scan_max) * 8);
    take(ws.row_ent, (size_t)std::max<uint64_t>(capacity, 1) * 8);
    take(ws.counts2, (size_t)std::max<uint64_t>(counts2_cap, 1) * 4);
    take(ws.values, (size_t)std::max<uint64_t>(capacity, 1) * 4);
    take(ws.tile_cost, (size_t)std::max<int64_t>(T, 1) * 4);
    take(ws.tile_order, (size_t)std::max<int64_t>(T, 1) * 4);
    return off;
}

// The device-table entry of one view; tile_base / row_base follow the views
// before it.
ViewParams make_view(const gs_camera* cam, int32_t width, int32_t height, float* out_rgb, float* out_T,
                     uint32_t* out_nc, uint32_t tile_base, uint32_t row_base)
{
    ViewParams v{};
    for (int k = 0; k < 9; ++k) v.R[k] = cam->R[k];
    for (int k = 0; k < 3; ++k) v.t[k] = cam->t[k];
    v.fx = cam->fx;
    v.fy = cam->fy;
    v.cx = cam->cx;
    v.cy = cam->cy;
    v.near_plane = cam->near_plane;
    for (int k = 0; k < 3; ++k)   // camera centre -R^T t
        v.campos[k] = (float)-(v.R[k] * v.t[0] + v.R[3 + k] * v.t[1] + v.R[6 + k] * v.t[2]);
    v.width = width;
    v.height = height;
    v.tiles_x = (width + kTile - 1) / kTile;
    v.tiles_y = (height + kTile - 1) / kTile;
    v.tile_base = tile_base;
    v.row_base = row_base;
    v.out_rgb = out_rgb;
    v.out_T = out_T;
    v.out_nc = out_nc;
    return v;
}

}  // namespace

extern "C" {

gs_status gs_create(int device, gs_context** out)
{
    if (!out) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "no such device");
    gs_context* ctx = new gs_context();
    ctx->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&ctx->host_info),
                          sizeof(uint32_t) * ((size_t)kMaxViews * kViewCounters + 16));
    // the pinned buffer is mapped into the device's address space: the
    // kernel that packs the frame's sizes writes them there, with no copy
    // (where it is not mapped, the sizes go through a device buffer and a
    // copy)
    if (e == hipSuccess &&
        hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->host_info_dev), ctx->host_info, 0) != hipSuccess) {
        (void)hipGetLastError();
        ctx->host_info_dev = nullptr;
    }
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ctx->noalloc_info), 64);
    // the device's copy of the no-allocation scratch (once per device)
    if (e == hipSuccess) e = init_scratch_address(device, count);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->sizes_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (ctx->sizes_ev) (void)hipEventDestroy(ctx->sizes_ev);
        if (ctx->host_info) (void)hipHostFree(ctx->host_info);
        if (ctx->noalloc_info) (void)hipFree(ctx->noalloc_info);
        delete ctx;
        return hip_fail(nullptr, e, "context set-up");
    }
    *out = ctx;
    return GS_OK;
}

void gs_destroy(gs_context* ctx)
{
    if (!ctx) return;
    if (ctx->graph) gs_graph_destroy(ctx->graph);
    (void)hipSetDevice(ctx->device);
    DevBuf* bufs[] = {&ctx->grad2d, &ctx->back_views, &ctx->ws.splats, &ctx->ws.depth_key, &ctx->ws.radius, &ctx->ws.tiles_touched, &ctx->ws.rect,
                      &ctx->ws.sort_ka, &ctx->ws.sort_va, &ctx->ws.sort_kb, &ctx->ws.sort_vb, &ctx->ws.hist,
                      &ctx->ws.scan_scratch, &ctx->ws.bin_info, &ctx->ws.counts1, &ctx->ws.rows_off, &ctx->ws.row_ent,
                      &ctx->ws.counts2, &ctx->ws.partials, &ctx->ws.views, &ctx->ws.row_tiles_x, &ctx->ws.view_counts,
                      &ctx->ws.counters, &ctx->ws.tile_offsets, &ctx->ws.values, &ctx->ws.tile_work, &ctx->ws.sorted_rect,
                      &ctx->ws.reuse_words, &ctx->ws.readback, &ctx->ws.tile_cost, &ctx->ws.tile_order,
                      &ctx->ws.sort_pa, &ctx->ws.sort_pb};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->host_info) (void)hipHostFree(ctx->host_info);
    if (ctx->noalloc_info) (void)hipFree(ctx->noalloc_info);
    for (hipEvent_t e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->sizes_ev) (void)hipEventDestroy(ctx->sizes_ev);
    delete ctx;
}

const char* gs_last_error(const gs_context* ctx)
{
    return ctx ? ctx->err.c_str() : g_thread_error.c_str();
}

gs_status gs_validate(const gs_gaussians* g, const gs_camera* cam, int32_t width, int32_t height,
                      const gs_render_opts* opts, const float* out_rgb)
{
    return validate(nullptr, g, cam, width, height, opts, out_rgb);
}

gs_status gs_render(gs_context* ctx, const gs_gaussians* g, const gs_camera* cam, int32_t width, int32_t height,
                    const gs_render_opts* opts, float* out_rgb, float* out_final_T, uint32_t* out_n_contrib,
                    void* stream)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (ctx->graph) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the context is bound to a render graph");
    gs_status st = validate(ctx, g, cam, width, height, opts, out_rgb);
    if (st != GS_OK) return st;
    std::vector<ViewParams> hv(1, make_view(cam, width, height, out_rgb, out_final_T, out_n_contrib, 0u, 0u));
    return render_views(ctx, g, hv, opts, static_cast<hipStream_t>(stream));
}

gs_status gs_render_noalloc(gs_context* ctx, const gs_gaussians* g, const gs_camera* cam, int32_t width, int32_t height,
                            const gs_render_opts* opts, float* out_rgb, float* out_final_T, uint32_t* out_n_contrib,
                            void* stream)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (ctx->graph) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the context is bound to a render graph");
    gs_status st = validate(ctx, g, cam, width, height, opts, out_rgb);
    if (st != GS_OK) return st;
    unsigned char* base = static_cast<unsigned char*>(scratch_address(ctx->device));
    if (!base) return fail(ctx, GS_ERR_HIP, "the device's no-allocation scratch has no address");
    std::vector<ViewParams> hv(1, make_view(cam, width, height, out_rgb, out_final_T, out_n_contrib, 0u, 0u));
    const Tuning tu = ctx->tuning;
    uint64_t cap = opts ? opts->pair_capacity : 0;
    if (cap > 0xFFFFFFFFull) return fail(ctx, GS_ERR_CAPACITY, "pair_capacity must stay below 2^32");
    if (cap == 0) {
        // the largest capacity whose buffers fit beside the scene's
        if (carve_noalloc(nullptr, nullptr, g->n, hv, tu, 1) > kNoallocScratchBytes)
            return fail(ctx, GS_ERR_CAPACITY,
                        "the scene's buffers exceed the no-allocation scratch of " +
                            std::to_string(kNoallocScratchBytes) + " bytes");
        uint64_t lo = 1, hi = 0xFFFFFFFFull;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo + 1) / 2;
            if (carve_noalloc(nullptr, nullptr, g->n, hv, tu, mid) <= kNoallocScratchBytes) lo = mid;
            else hi = mid - 1;
        }
        cap = lo;
    }
    const size_t need = carve_noalloc(nullptr, nullptr, g->n, hv, tu, cap);
    if (need > kNoallocScratchBytes)
        return fail(ctx, GS_ERR_CAPACITY,
                    "a render of this size needs " + std::to_string(need) + " bytes; the no-allocation scratch holds " +
                        std::to_string(kNoallocScratchBytes));
    Workspace fw;
    carve_noalloc(&fw, base, g->n, hv, tu, cap);
    gs_render_opts o{};
    o.tile_size = kTile;
    if (opts) o = *opts;
    o.pair_capacity = cap;
    o.flags &= ~GS_RENDER_REUSE_ORDER;
    return render_views(ctx, g, hv, &o, static_cast<hipStream_t>(stream), true, &fw);
}

gs_status gs_render_batched(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                            const gs_render_opts* opts, void* stream)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (ctx->graph) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the context is bound to a render graph");
    std::vector<ViewParams> hv;
    gs_status st = build_views(ctx, g, views, n_views, opts, hv);
    if (st != GS_OK) return st;
    return render_views(ctx, g, hv, opts, static_cast<hipStream_t>(stream));
}

gs_status gs_graph_create(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                          const gs_render_opts* opts, void* stream, gs_graph** out)
{
    if (!ctx || !out) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    *out = nullptr;
    if (ctx->graph) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the context is bound to a render graph");
    if (!opts || opts->pair_capacity == 0)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "a render graph needs opts->pair_capacity > 0");
    std::vector<ViewParams> hv;
    gs_status st = build_views(ctx, g, views, n_views, opts, hv);
    if (st != GS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // an eager render sizes every buffer (capture must not allocate) and
    // writes the view table
    if ((st = render_views(ctx, g, hv, opts, s)) != GS_OK) return st;
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    gs_graph* gr = new gs_graph();
    gr->ctx = ctx;
    gr->views = hv;
    hipError_t e = hipStreamCreateWithFlags(&gr->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(gr->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        if (gr->capture) (void)hipStreamDestroy(gr->capture);
        delete gr;
        return hip_fail(ctx, e, "begin capture");
    }
    const uint32_t profiling = ctx->profiling;
    ctx->profiling = 0;   // no event records inside the graph
    st = render_views(ctx, g, hv, opts, gr->capture, false);
    ctx->profiling = profiling;
    e = hipStreamEndCapture(gr->capture, &gr->graph);
    if (st == GS_OK && e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (st != GS_OK || e != hipSuccess) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        (void)hipStreamDestroy(gr->capture);
        delete gr;
        return st != GS_OK ? st : hip_fail(ctx, e, "capture");
    }
    ctx->graph = gr;
    *out = gr;
    return GS_OK;
}

gs_status gs_graph_set_views(gs_graph* graph, const gs_view* views, int32_t n_views, void* stream)
{
    if (!graph) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "graph is NULL");
    gs_context* ctx = graph->ctx;
    if (!views || n_views != (int32_t)graph->views.size())
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "n_views must equal the captured view count");
    std::vector<ViewParams> hv = graph->views;
    for (int v = 0; v < n_views; ++v) {
        const gs_view& w = views[v];
        gs_status st = validate_view(ctx, &w.camera, w.width, w.height, w.out_rgb);
        if (st != GS_OK) return st;
        if (w.width != hv[v].width || w.height != hv[v].height)
            return fail(ctx, GS_ERR_INVALID_ARGUMENT, "view sizes must equal the captured ones");
        hv[v] = make_view(&w.camera, w.width, w.height, w.out_rgb, w.out_final_T, w.out_n_contrib, hv[v].tile_base,
                          hv[v].row_base);
    }
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(write_view_table(hv, static_cast<ViewParams*>(ctx->ws.views.p), static_cast<hipStream_t>(stream)),
            "view table");
    graph->views = hv;
    return GS_OK;
}

gs_status gs_graph_launch(gs_graph* graph, void* stream)
{
    if (!graph) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "graph is NULL");
    gs_context* ctx = graph->ctx;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
    ctx->stream = static_cast<hipStream_t>(stream);
    // the launch rendered the graph's current cameras into its current
    // outputs: a backward now differentiates that render
    ctx->last_views = graph->views;
    ctx->have_render = true;
    ctx->timed = false;
    ctx->traced = false;
    return GS_OK;
}

void gs_graph_destroy(gs_graph* graph)
{
    if (!graph) return;
    (void)hipSetDevice(graph->ctx->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    if (graph->capture) (void)hipStreamDestroy(graph->capture);
    if (graph->ctx->graph == graph) graph->ctx->graph = nullptr;
    delete graph;
}

}  // extern "C"

namespace {

// Validated views of a batched render with their tile and row bases.
gs_status build_views(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                      const gs_render_opts* opts, std::vector<ViewParams>& hv)
{
    gs_status st = validate_gaussians(ctx, g);
    if (st == GS_OK) st = validate_opts(ctx, opts);
    if (st != GS_OK) return st;
    if (!views) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "views is NULL");
    if (n_views < 1 || n_views > kMaxViews) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "n_views must lie in [1, 1024]");
    if ((int64_t)n_views * g->n > 0xFFFFFFFFll)
        return fail(ctx, GS_ERR_UNSUPPORTED, "n_views * n must stay below 2^32");
    hv.clear();
    hv.reserve((size_t)n_views);
    int64_t tile_base = 0, row_base = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_view& w = views[v];
        if ((st = validate_view(ctx, &w.camera, w.width, w.height, w.out_rgb)) != GS_OK) return st;
        hv.push_back(make_view(&w.camera, w.width, w.height, w.out_rgb, w.out_final_T, w.out_n_contrib,
                               (uint32_t)tile_base, (uint32_t)row_base));
        tile_base += (int64_t)hv.back().tiles_x * hv.back().tiles_y;
        row_base += hv.back().tiles_y;
        if (row_base > kMaxTotalRows) return fail(ctx, GS_ERR_UNSUPPORTED, "more than 16384 tile rows over all views");
        if (tile_base >= (int64_t(1) << 31)) return fail(ctx, GS_ERR_UNSUPPORTED, "too many tiles over all views");
    }
    return GS_OK;
}

}  // namespace

extern "C" {

gs_status gs_render_backward(gs_context* ctx, const gs_gaussians* g, const float* const* grad_rgb,
                             const float* const* grad_final_T, const gs_gradients* grads, void* stream)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!g || !grad_rgb || !grads) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!ctx->have_render) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "no render on this context yet");
    const gs_gaussians& f = ctx->last_g;
    if (g->n != f.n || g->sh_degree != f.sh_degree || g->attr_dtype != f.attr_dtype || g->means != f.means ||
        g->log_scales != f.log_scales || g->quats != f.quats || g->opacity_logits != f.opacity_logits ||
        g->sh != f.sh)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "g must be the scene of the last render on this context");
    if (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "a gradient pointer is NULL");
    std::vector<ViewParams> hv = ctx->last_views;
    const int V = (int)hv.size();
    for (int v = 0; v < V; ++v) {
        if (!hv[v].out_T || !hv[v].out_nc)
            return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the forward render must write out_final_T and out_n_contrib");
        if (!grad_rgb[v]) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "grad_rgb holds a NULL view");
        hv[v].grad_rgb = grad_rgb[v];
        hv[v].grad_T = grad_final_T ? grad_final_T[v] : nullptr;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    gs_status st;
    const int64_t items = ctx->n * V;
    if ((st = ensure(ctx, ctx->grad2d, (size_t)std::max<int64_t>(items, 1) * kGrad2d * 4)) != GS_OK) return st;
    if ((st = ensure(ctx, ctx->back_views, (size_t)V * sizeof(ViewParams))) != GS_OK) return st;
    // a table of its own: the render's table stays as a captured graph reads it
    ViewParams* views = static_cast<ViewParams*>(ctx->back_views.p);
    HIP_TRY(write_view_table(hv, views, s), "view table");
    float* grad2d = static_cast<float*>(ctx->grad2d.p);
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, items * kGrad2d, s), "clear gradients");
    BlendBackArgs bb{};
    bb.splats = static_cast<const Splat*>(ctx->ws.splats.p);
    bb.values = static_cast<const uint32_t*>(ctx->ws.values.p);
    bb.tile_offsets = static_cast<const uint32_t*>(ctx->ws.tile_offsets.p);
    bb.views = views;
    bb.n_views = V;
    bb.tiles = ctx->tiles;
    bb.group = ctx->last_tuning.blend_group;
    // the forward's dispatch order (its buffer is rewritten only by a forward)
    bb.order = bb.group <= 0 ? static_cast<const uint32_t*>(ctx->ws.tile_order.p) : nullptr;
    for (int k = 0; k < 3; ++k) bb.bg[k] = ctx->last_bg[k];
    bb.grad2d = grad2d;
    HIP_TRY(launch_blend_backward(bb, ctx->capacity, s), "blend backward");
    ProjectBackArgs pb{};
    pb.n = g->n;
    pb.sh_degree = g->sh_degree;
    pb.dtype = g->attr_dtype;
    pb.means = g->means;
    pb.log_scales = g->log_scales;
    pb.quats = g->quats;
    pb.logits = g->opacity_logits;
    pb.sh = g->sh;
    pb.views = views;
    pb.n_views = V;
    pb.grad2d = grad2d;
    pb.tiles_touched = static_cast<const uint32_t*>(ctx->ws.tiles_touched.p);
    pb.g_means = grads->means;
    pb.g_log_scales = grads->log_scales;
    pb.g_quats = grads->quats;
    pb.g_logits = grads->opacity_logits;
    pb.g_sh = grads->sh;
    HIP_TRY(launch_project_backward(pb, s), "projection backward");
    ctx->stream = s;
    return GS_OK;
}

gs_status gs_get_order_reuse(gs_context* ctx, uint32_t* out2)
{
    if (!ctx || !out2) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!ctx->have_render || !ctx->last_reuse)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the last render did not start from the previous order");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    uint32_t w[kReuseWords];
    HIP_TRY(hipMemcpyAsync(w, ctx->ws.reuse_words.p, sizeof w, hipMemcpyDeviceToHost, ctx->stream), "read reuse words");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    out2[0] = w[0];
    out2[1] = w[1];
    return GS_OK;
}

gs_status gs_get_list_reuse(gs_context* ctx, uint32_t* out2)
{
    if (!ctx || !out2) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!ctx->have_render || !ctx->lists_compared)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the last render did not compare its keys and rectangles");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    uint32_t w[2];
    HIP_TRY(hipMemcpyAsync(w, static_cast<uint32_t*>(ctx->ws.counters.p) + kCounterChanged, sizeof w,
                           hipMemcpyDeviceToHost, ctx->stream),
            "read list reuse words");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    out2[0] = w[1];
    out2[1] = w[0];
    return GS_OK;
}

gs_status gs_get_list_info(gs_context* ctx, gs_list_info* out)
{
    if (!ctx || !out) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (ctx->last_noalloc) {
        // sizes a no-allocation render packed: view counters, the counters,
        // R, level-2 sizes
        HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
        uint32_t w[kViewCounters + 7];
        HIP_TRY(hipMemcpyAsync(w, ctx->noalloc_info, sizeof w, hipMemcpyDeviceToHost, ctx->stream), "read sizes");
        HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        const uint64_t K = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
        out->num_pairs = K;
        out->num_row_entries = w[kViewCounters + 4];
        out->tiles_x = ctx->tiles_x;
        out->tiles_y = ctx->tiles_y;
        out->n_visible = (int64_t)w[0];
        out->num_tiles = ctx->tiles;
        out->num_views = ctx->n_views;
        if (w[kViewCounters + 1] != 0 || K > ctx->capacity)
            return fail(ctx, GS_ERR_CAPACITY, "the last render produced more pairs than pair_capacity");
        return GS_OK;
    }
    if (!ctx->have_render) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "no render on this context yet");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    std::vector<uint32_t> vc((size_t)ctx->n_views * kViewCounters);
    uint32_t c[4], r32 = 0;
    HIP_TRY(hipMemcpyAsync(vc.data(), ctx->ws.view_counts.p, vc.size() * 4, hipMemcpyDeviceToHost, ctx->stream),
            "read view counts");
    HIP_TRY(hipMemcpyAsync(c, ctx->ws.counters.p, sizeof c, hipMemcpyDeviceToHost, ctx->stream), "read counters");
    HIP_TRY(hipMemcpyAsync(&r32, static_cast<uint32_t*>(ctx->ws.rows_off.p) + ctx->rows, sizeof r32,
                           hipMemcpyDeviceToHost, ctx->stream),
            "read R");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    uint64_t K = 0, vis = 0;
    for (int v = 0; v < ctx->n_views; ++v) {
        vis += vc[(size_t)v * kViewCounters];
        K += (uint64_t)vc[(size_t)v * kViewCounters + 2] | ((uint64_t)vc[(size_t)v * kViewCounters + 3] << 32);
    }
    const uint64_t R = r32;
    out->num_pairs = K;
    out->num_row_entries = R;
    out->tiles_x = ctx->tiles_x;
    out->tiles_y = ctx->tiles_y;
    out->n_visible = (int64_t)vis;
    out->num_tiles = ctx->tiles;
    out->num_views = ctx->n_views;
    if (c[1] != 0 || K > ctx->capacity || R > K)
        return fail(ctx, GS_ERR_CAPACITY, "the last render produced more pairs than pair_capacity");
    return GS_OK;
}

gs_status gs_copy_lists(gs_context* ctx, uint32_t* values, uint32_t* tile_offsets, uint64_t* keys, void* stream)
{
    if (ctx && ctx->last_noalloc)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the lists of a no-allocation render are not kept");
    gs_list_info info;
    gs_status st = gs_get_list_info(ctx, &info);
    if (st != GS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t T = ctx->tiles;
    if (values && info.num_pairs)
        HIP_TRY(hipMemcpyAsync(values, ctx->ws.values.p, info.num_pairs * 4, hipMemcpyDeviceToDevice, s), "copy values");
    if (tile_offsets)
        HIP_TRY(hipMemcpyAsync(tile_offsets, ctx->ws.tile_offsets.p, (size_t)(T + 1) * 4, hipMemcpyDeviceToDevice, s),
                "copy offsets");
    if (keys)
        HIP_TRY(launch_write_keys(static_cast<const uint32_t*>(ctx->ws.values.p),
                                  static_cast<const uint32_t*>(ctx->ws.tile_offsets.p),
                                  static_cast<const uint32_t*>(ctx->ws.depth_key.p), T, keys, s),
                "write keys");
    return GS_OK;
}

gs_status gs_copy_projection(gs_context* ctx, float* splats, uint32_t* depth_key, int32_t* radius,
                             uint32_t* tiles_touched, uint16_t* rect, void* stream)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!ctx->have_render) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "no render on this context yet");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)ctx->n * (size_t)ctx->n_views;
    if (n == 0) return GS_OK;
    if (splats) HIP_TRY(hipMemcpyAsync(splats, ctx->ws.splats.p, n * sizeof(Splat), hipMemcpyDeviceToDevice, s), "copy");
    if (depth_key) HIP_TRY(hipMemcpyAsync(depth_key, ctx->ws.depth_key.p, n * 4, hipMemcpyDeviceToDevice, s), "copy");
    if (radius) HIP_TRY(hipMemcpyAsync(radius, ctx->ws.radius.p, n * 4, hipMemcpyDeviceToDevice, s), "copy");
    if (tiles_touched)
        HIP_TRY(hipMemcpyAsync(tiles_touched, ctx->ws.tiles_touched.p, n * 4, hipMemcpyDeviceToDevice, s), "copy");
    if (rect) HIP_TRY(hipMemcpyAsync(rect, ctx->ws.rect.p, n * 8, hipMemcpyDeviceToDevice, s), "copy");
    return GS_OK;
}

gs_status gs_set_profiling(gs_context* ctx, int32_t flags)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (flags & ~(GS_PROFILE_STAGES | GS_PROFILE_BLEND_WORK))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "unknown profiling flag");
    if ((flags & GS_PROFILE_STAGES) && !ctx->ev[0]) {
        HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
        for (hipEvent_t& e : ctx->ev) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    }
    ctx->profiling = (uint32_t)flags;
    return GS_OK;
}

gs_status gs_get_stage_times(gs_context* ctx, float* ms, int32_t count)
{
    if (!ctx || !ms) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (count != GS_NUM_STAGES) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "count must be GS_NUM_STAGES");
    if (!(ctx->have_render || ctx->last_noalloc) || !ctx->timed)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the last render was not timed (gs_set_profiling)");
    HIP_TRY(hipEventSynchronize(ctx->ev[8]), "hipEventSynchronize");
    const int from[GS_NUM_STAGES] = {0, 1, 2, 4, 5, 6, 7};
    const int to[GS_NUM_STAGES] = {1, 2, 3, 5, 6, 7, 8};
    for (int k = 0; k < GS_NUM_STAGES; ++k)
        HIP_TRY(hipEventElapsedTime(&ms[k], ctx->ev[from[k]], ctx->ev[to[k]]), "hipEventElapsedTime");
    return GS_OK;
}

namespace {

Tuning from_abi(const gs_tuning& t)
{
    return Tuning{t.sort_items, t.bin_row_items, t.bin_tile_items, t.blend_tile_group, t.blend_batch};
}

gs_tuning to_abi(const Tuning& t)
{
    gs_tuning o;
    o.sort_items = t.sort_items;
    o.bin_row_items = t.bin1_items;
    o.bin_tile_items = t.bin2_items;
    o.blend_tile_group = t.blend_group;
    o.blend_batch = t.blend_batch;
    return o;
}

// The candidates gs_autotune tries, in the order of its out_ms array: each
// parameter of Tuning with the stages whose time scores it (indices
// into the GS_NUM_STAGES stage times).
struct TuneParam {
    int Tuning::*field;
    int values[9];
    int count;
    int stage_lo, stage_hi;   // stages [lo, hi]
};
const TuneParam kTuneParams[] = {
    {&Tuning::sort_items, {4, 8, 16}, 3, 1, 1},
    {&Tuning::bin1_items, {4, 8, 16}, 3, 2, 5},
    {&Tuning::bin2_items, {8, 16, 32}, 3, 2, 5},
    {&Tuning::blend_group, {-1, 0, 1, 2, 4, 8, 16, 32, 64}, 9, 6, 6},
    {&Tuning::blend_batch, {128, 256, 512}, 3, 6, 6},
};

}  // namespace

gs_status gs_set_tuning(gs_context* ctx, const gs_tuning* tuning)
{
    if (!ctx || !tuning) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    const Tuning t = from_abi(*tuning);
    if (!tuning_supported(t))
        return fail(ctx, GS_ERR_INVALID_ARGUMENT,
                    "unsupported tuning: sort_items and bin_row_items take 4, 8 or 16, bin_tile_items 8, 16 or 32, "
                    "blend_tile_group -1..64, blend_batch 128, 256 or 512");
    ctx->tuning = t;
    return GS_OK;
}

gs_status gs_get_tuning(gs_context* ctx, gs_tuning* out)
{
    if (!ctx || !out) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    *out = to_abi(ctx->tuning);
    return GS_OK;
}

gs_status gs_autotune(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                      const gs_render_opts* opts, int32_t reps, void* stream, gs_tuning* out, float* out_ms)
{
    if (!ctx) return fail(nullptr, GS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (ctx->graph) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the context is bound to a render graph");
    if (reps < 1 || reps > 1000) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "reps must lie in [1, 1000]");
    std::vector<ViewParams> hv;
    gs_status st = build_views(ctx, g, views, n_views, opts, hv);
    if (st != GS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t saved_flags = ctx->profiling;
    const Tuning start = ctx->tuning;
    Tuning cur = start;
    if ((st = gs_set_profiling(ctx, GS_PROFILE_STAGES)) != GS_OK) return st;   // creates the stage events
    int k_out = 0;
    for (const TuneParam& p : kTuneParams) {
        float best_ms = INFINITY;
        int best = cur.*p.field;
        for (int c = 0; c < p.count; ++c) {
            Tuning t = cur;
            t.*p.field = p.values[c];
            ctx->tuning = t;
            float sum = 0.f;
            // one untimed render sizes the buffers this shape needs
            for (int r = 0; r <= reps && st == GS_OK; ++r) {
                st = render_views(ctx, g, hv, opts, s);
                float ms[GS_NUM_STAGES];
                if (st == GS_OK) st = gs_get_stage_times(ctx, ms, GS_NUM_STAGES);
                if (st == GS_OK && r > 0)
                    for (int k = p.stage_lo; k <= p.stage_hi; ++k) sum += ms[k];
            }
            if (st != GS_OK) {
                ctx->tuning = start;
                ctx->profiling = saved_flags;
                return st;
            }
            const float avg = sum / (float)reps;
            if (out_ms) out_ms[k_out] = avg;
            ++k_out;
            if (avg < best_ms) {
                best_ms = avg;
                best = p.values[c];
            }
        }
        cur.*p.field = best;
    }
    ctx->tuning = cur;
    ctx->profiling = saved_flags;
    if (out) *out = to_abi(cur);
    return GS_OK;
}

namespace {
gs_status read_tile_work(gs_context* ctx, std::vector<uint64_t>& w)
{
    if (!ctx->have_render || !ctx->traced)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "the last render did not count blend work (GS_PROFILE_BLEND_WORK)");
    const size_t T = (size_t)ctx->tiles;
    w.assign(T * kTileWorkFields, 0);
    if (T == 0) return GS_OK;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(w.data(), ctx->ws.tile_work.p, T * kTileWorkFields * 8, hipMemcpyDeviceToHost, ctx->stream),
            "read tile work");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return GS_OK;
}
}  // namespace

gs_status gs_get_blend_stats(gs_context* ctx, uint64_t* stats4)
{
    if (!ctx || !stats4) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    std::vector<uint64_t> w;
    gs_status st = read_tile_work(ctx, w);
    if (st != GS_OK) return st;
    uint64_t ev = 0, co = 0, staged = 0, bodies = 0;
    for (size_t t = 0; t * kTileWorkFields < w.size(); ++t) {
        const uint64_t* r = w.data() + t * kTileWorkFields;
        staged += r[2];
        bodies += r[3];
        ev += r[4];
        co += r[5];
    }
    stats4[0] = ev;
    stats4[1] = co;
    stats4[2] = staged;
    stats4[3] = 64 * bodies;
    return GS_OK;
}

gs_status gs_get_blend_tile_work(gs_context* ctx, uint64_t* work, int64_t tiles)
{
    if (!ctx || !work) return fail(ctx, GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!ctx->have_render || tiles != ctx->tiles)
        return fail(ctx, GS_ERR_INVALID_ARGUMENT, "tiles must be the tile count of the last render");
    std::vector<uint64_t> w;
    gs_status st = read_tile_work(ctx, w);
    if (st != GS_OK) return st;
    std::memcpy(work, w.data(), w.size() * sizeof(uint64_t));
    return GS_OK;
}

}  // extern "C"
