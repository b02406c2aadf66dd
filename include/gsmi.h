/*
 * gsmi.h -- C ABI of the MI355X (gfx950) 3D Gaussian Splatting forward
 * rasterizer.
 *
 * The library renders one image of a set of 3D Gaussians (Sec. 3.1 of
 * "Rendering 3D Gaussians on a Graph Processor"): it culls and projects every
 * Gaussian (EWA splatting, Sigma' = J W Sigma W^T J^T, SH colour), bins each
 * one into 64-bit (tile << 32 | depth) keys over 16x16-pixel screen tiles
 * using the 3-sigma square bound of Sec. 4.4, sorts the keys, and composites
 * every pixel front to back with Eq. 1 and early termination.
 *
 * Conventions
 *   - Every array pointer in this header is a DEVICE pointer (HIP device
 *     memory of the context's device) owned by the caller, unless a comment
 *     says otherwise.  Structures themselves are read on the host.
 *   - Arrays are structure-of-arrays, channel-major: element (c, i) of an
 *     array declared [C][n] lives at index c*n + i.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued on it; gs_render blocks the host once per call to
 *     read the pair count (see pair_capacity).
 *   - A context is not thread-safe: use one per host thread / stream.
 *   - Errors: every argument is checked on the host before anything is
 *     enqueued; on an error return no output has been written.
 *     gs_last_error() gives a message for the last failing call on a context
 *     (or on the calling thread when the context pointer was NULL).
 */
#ifndef GSMI_H
#define GSMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size, degree, camera, option */
    GS_ERR_OUT_OF_MEMORY = 2,    /* device allocation of the workspace failed */
    GS_ERR_CAPACITY = 3,         /* more (Gaussian, tile) pairs than allowed */
    GS_ERR_HIP = 4,              /* a HIP runtime call failed (message says which) */
    GS_ERR_UNSUPPORTED = 5       /* valid request outside what the library supports */
} gs_status;

typedef enum { GS_F32 = 0, GS_BF16 = 1, GS_F16 = 2 } gs_dtype;

typedef struct gs_context gs_context;

/* Gaussians of the scene (Sec. 3.1: mean, rotation and scale of the
 * covariance Sigma = R S S^T R^T, opacity, SH colour; the record of Sec. 4.5
 * stores scale in log space and rotation as a quaternion).
 *   n               number of Gaussians, 0 <= n < 2^31
 *   sh_degree       0..3; (sh_degree+1)^2 coefficients per colour channel
 *   attr_dtype      storage type of log_scales, quats, opacity_logits and sh
 *                   (means are always float32)
 *   means           float [3][n]  world-space centres
 *   log_scales      [3][n]        per-axis log standard deviation
 *   quats           [4][n]        rotation quaternion (w, x, y, z); it is
 *                                 normalised by the renderer; a zero
 *                                 quaternion culls the Gaussian
 *   opacity_logits  [n]           opacity before the logistic sigmoid
 *   sh              [(deg+1)^2][3][n]  real SH coefficients, index
 *                                 k = l*l + l + m (m = -l..l), then channel */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t attr_dtype;
    const float* means;
    const void* log_scales;
    const void* quats;
    const void* opacity_logits;
    const void* sh;
} gs_gaussians;

/* Pinhole camera.  R (row-major) and t map world to camera coordinates,
 * x right, y down, z forward; a camera-space point (x, y, z) lands on the
 * image point (fx x/z + cx, fy y/z + cy), and pixel (px, py) samples the
 * image point (px, py).  Gaussians with camera-space z <= near_plane are
 * culled (Sec. 4.5).  All values must be finite; fx, fy, near_plane > 0. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float near_plane;
} gs_camera;

/* Render options.
 *   background     colour added with the final transmittance
 *   tile_size      must be 16
 *   pair_capacity  0: the library reads the pair count back to the host
 *                  and grows its buffers (one host sync per render);
 *                  > 0: fixed upper bound on (Gaussian, tile) pairs and no
 *                  host sync; pairs past the bound are dropped without any
 *                  out-of-bounds write, the image is then unspecified, and
 *                  gs_get_list_info (hence gs_copy_lists) returns
 *                  GS_ERR_CAPACITY for that render; above 2^32 - 1:
 *                  GS_ERR_UNSUPPORTED (pair offsets are 32-bit; a render
 *                  with more pairs returns GS_ERR_CAPACITY after the row
 *                  counts, before the pair buffers are sized or any output
 *                  is written)
 *   flags          0, GS_RENDER_REUSE_ORDER or GS_RENDER_REUSE_LISTS
 *                  (below), or both; other bits give GS_ERR_INVALID_ARGUMENT */
typedef struct {
    float background[3];
    int32_t tile_size;
    uint64_t pair_capacity;
    uint32_t flags;
} gs_render_opts;

/* GS_RENDER_REUSE_ORDER: frame-to-frame reuse of the depth order, after the
 * data locality of Sec. 5.7 (Table 5).  When the previous render on the
 * context was a single view of as many Gaussians, the depth sort first
 * re-keys that render's order with this frame's depths and counts the
 * adjacent pairs it puts out of order.  None (a static camera, changes of
 * colour or opacity only): the radix sort is skipped.  At most n/256: runs
 * of 8192 are sorted in on-chip memory twice (the second time shifted by
 * half a run) and, if the result checks out on the device, the radix sort is
 * skipped.  Otherwise the radix sort runs as usual.  The order, hence every
 * output, is the same as without the flag; only the time differs.  Ignored
 * for batched renders and for the first render on a context. */
#define GS_RENDER_REUSE_ORDER 1u

/* GS_RENDER_REUSE_LISTS: frame-to-frame reuse of the whole tile lists, the
 * case of Sec. 5.7 (Table 5) where no Gaussian changes its tiles.  The lists
 * of Sec. 3.1 depend only on the depth keys, the tile rectangles and the
 * image size.  When the previous render on the context rendered as many
 * Gaussians in as many views of the same widths and heights, with the same
 * pair_capacity (0 included), the projection compares each (view, Gaussian)
 * item's depth key and rectangle with that render's and counts those that
 * differ.  None (a static camera; colour, SH
 * or opacity edits): every kernel of the depth sort and the binning finds
 * that on the device and does nothing, and the blend reads the lists kept
 * in the context, which are the ones this frame would build.  Otherwise the
 * render goes on as usual (with GS_RENDER_REUSE_ORDER, trying the order).
 * The decision needs no host read, so a captured graph can carry the flag.
 * Every output is the same as without the flag.  Applies to gs_render,
 * gs_render_batched and graphs alike; ignored for the first render on a
 * context; gs_get_list_reuse reports the outcome. */
#define GS_RENDER_REUSE_LISTS 2u

/* Creates a context on HIP device `device`; *out receives it. */
gs_status gs_create(int device, gs_context** out);

/* Frees the context and its workspace; NULL is allowed. */
void gs_destroy(gs_context* ctx);

/* Message of the last failing call on ctx (NULL: on this thread).  The
 * string is owned by the library and valid until the next call. */
const char* gs_last_error(const gs_context* ctx);

/* Checks every argument of gs_render without touching a device; returns
 * the status gs_render would return for them before enqueuing anything. */
gs_status gs_validate(const gs_gaussians* g, const gs_camera* cam, int32_t width, int32_t height,
                      const gs_render_opts* opts, const float* out_rgb);

/* Renders one image (Sec. 3.1 stages 1-4, Eq. 1).
 *   width, height   image size in pixels, 1..32768 each
 *   out_rgb         float [3][height][width]; colour C + T * background,
 *                   not clamped
 *   out_final_T     float [height][width] final transmittance, or NULL
 *   out_n_contrib   uint32 [height][width], or NULL: one past the position
 *                   (within the pixel's tile list) of the last Gaussian that
 *                   contributed to the pixel, 0 if none
 * The per-tile lists and the projected Gaussians of this render stay in the
 * context until the next gs_render or gs_destroy (see below). */
gs_status gs_render(gs_context* ctx, const gs_gaussians* g, const gs_camera* cam,
                    int32_t width, int32_t height, const gs_render_opts* opts,
                    float* out_rgb, float* out_final_T, uint32_t* out_n_contrib, void* stream);

/* gs_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * renders what gs_render renders (same kernels, same bits) but takes every
 * buffer of the render from one static device array of 64 MiB per device
 * (held from library load to process end) and calls no hipMalloc, hipFree
 * or other allocating routine, and never synchronises the host.
 *   opts->pair_capacity  > 0: the bound on (Gaussian, tile) pairs, as for
 *                        gs_render; 0: the largest bound whose buffers fit
 *                        beside the scene's
 *   GS_ERR_CAPACITY      before any launch when the scene, image and
 *                        capacity need more than the 64 MiB (the message
 *                        gives the bytes needed); pairs past the capacity
 *                        are dropped on the device as for gs_render, which
 *                        gs_get_list_info reports afterwards
 * GS_RENDER_REUSE_ORDER, GS_RENDER_REUSE_LISTS and GS_PROFILE_BLEND_WORK
 * are ignored, and the blend takes no per-tile history (a heaviest-first order, if tuned, comes
 * from list lengths).  After it, gs_get_list_info and gs_get_stage_times
 * work; the lists, projection and backward of the render are not kept
 * (gs_copy_lists, gs_copy_projection and gs_render_backward fail).  Every
 * call on one device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (two streams, two threads, two
 * contexts) race and must be ordered by the caller. */
gs_status gs_render_noalloc(gs_context* ctx, const gs_gaussians* g, const gs_camera* cam,
                            int32_t width, int32_t height, const gs_render_opts* opts,
                            float* out_rgb, float* out_final_T, uint32_t* out_n_contrib, void* stream);

/* One view of a batched render: a camera, its image size and its outputs
 * (device memory owned by the caller, laid out as for gs_render). */
typedef struct {
    gs_camera camera;
    int32_t width, height;        /* 1..32768 each */
    float* out_rgb;               /* float [3][height][width] */
    float* out_final_T;           /* float [height][width], or NULL */
    uint32_t* out_n_contrib;      /* uint32 [height][width], or NULL */
} gs_view;

/* Renders n_views views of one scene in one call: the batched form of
 * gs_render (the same computation per view, Sec. 3.1 stages 1-4 and Eq. 1).
 * Every stage runs once over all views: each Gaussian's attributes are read
 * once and projected into every view; the depth sort sorts each view's
 * Gaussians (as one segmented sort); binning and blending run over the
 * concatenated tile grids of the views, so small and large images share the
 * launches.  Each view's image equals what gs_render returns for it alone.
 *   views     host array [n_views], 1 <= n_views <= 1024
 *   lists     the per-tile lists cover all views: global tile t indexes the
 *             views' row-major tile grids concatenated in view order, and a
 *             list holds items v * n + i (view v, Gaussian i); requires
 *             n_views * n < 2^32 and at most 16384 tile rows over all views
 *             (GS_ERR_UNSUPPORTED otherwise)
 * Errors as for gs_render, checked for every view before any launch. */
gs_status gs_render_batched(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                            const gs_render_opts* opts, void* stream);

/* A batched render captured once into a HIP graph and replayed: the
 * persistent form of gs_render_batched for callers that render the same set
 * of view sizes frame after frame (every kernel of the render in one graph
 * launch, no host round trip, no allocation).
 *
 * gs_graph_create renders once eagerly on `stream` (sizing the workspace
 * from opts->pair_capacity, which must be > 0: the graph cannot read the
 * pair count back), then captures the same render into a graph.  While the
 * graph exists the context belongs to it: gs_render and gs_render_batched
 * on ctx fail with GS_ERR_INVALID_ARGUMENT; the list and projection queries
 * work on the last launch.  The scene pointers in g must stay valid and may
 * change contents between launches.
 * gs_graph_set_views replaces the cameras and output pointers (same count
 * and sizes as at creation) by a small upload on `stream`; the next launch
 * renders them.
 * gs_graph_launch enqueues one render on `stream`; an overflow of
 * pair_capacity is reported by gs_get_list_info after it.  The flags of
 * opts act in every replay (their decisions are taken on the device):
 * GS_RENDER_REUSE_LISTS keeps the lists of the previous replay when no depth
 * key or rectangle changed.
 * gs_graph_destroy releases the graph and frees the context (NULL-safe). */
typedef struct gs_graph gs_graph;
gs_status gs_graph_create(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                          const gs_render_opts* opts, void* stream, gs_graph** out);
gs_status gs_graph_set_views(gs_graph* graph, const gs_view* views, int32_t n_views, void* stream);
gs_status gs_graph_launch(gs_graph* graph, void* stream);
void gs_graph_destroy(gs_graph* graph);

/* Gradients of a scalar loss with respect to the Gaussian parameters, float32
 * device arrays in the layouts of gs_gaussians (owned by the caller,
 * overwritten): means [3][n], log_scales [3][n], quats [4][n] (of the raw,
 * unnormalised quaternion), opacity_logits [n], sh [(deg+1)^2][3][n].  For
 * BF16/FP16 storage they are the gradients at the stored values. */
typedef struct {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} gs_gradients;

/* Backward of the last render on ctx (gs_render, gs_render_batched, or the
 * last gs_graph_launch of a graph on ctx, with the cameras and outputs that
 * launch rendered; the differentiable part of Sec. 3.1 stages 1, 2 and 4 --
 * the tile lists and
 * their order are held fixed, as are the 3-sigma rectangles): given
 * dL/d(out_rgb) per view and optionally dL/d(out_final_T), writes dL/d(the
 * Gaussian parameters) into grads.  The blend is recomputed front to back
 * from the forward's own outputs (out_rgb, out_final_T, out_n_contrib of every
 * view, which must have been requested and still hold that render's values)
 * rather than stored; the alpha threshold, the 0.99 clamp and the early
 * termination pass no gradient, nor does a colour clamped at 0.
 *   g             the scene of that render (same pointers)
 *   grad_rgb      host array [n_views] of device pointers, float [3][H][W]
 *   grad_final_T  NULL, or host array [n_views] of device pointers (each
 *                 float [H][W] or NULL)
 * GS_ERR_INVALID_ARGUMENT when g differs from the last render's scene, an
 * output of that render was not kept, or a pointer is NULL. */
gs_status gs_render_backward(gs_context* ctx, const gs_gaussians* g, const float* const* grad_rgb,
                             const float* const* grad_final_T, const gs_gradients* grads, void* stream);

/* Sizes of the last render's per-tile lists (host values; synchronises the
 * context's last stream). */
typedef struct {
    uint64_t num_pairs;        /* K, total (Gaussian, tile) pairs */
    int32_t tiles_x, tiles_y;
    int64_t n_visible;         /* Gaussians overlapping at least one tile */
    uint64_t num_row_entries;  /* (Gaussian, tile row) pairs of the binning */
    int64_t num_tiles;         /* tiles over all views (tiles_x * tiles_y for one view) */
    int32_t num_views;         /* views of the last render */
} gs_list_info;

gs_status gs_get_list_info(gs_context* ctx, gs_list_info* out);

/* Copies the last render's per-tile lists into caller memory: the output of
 * the duplicate-and-sort stages of Sec. 3.1 (every (Gaussian, tile) pair,
 * ordered by the 64-bit key tile << 32 | depth), which the blend walks.
 * Device pointers on the context's device, written on `stream`; the caller
 * sizes them from gs_get_list_info, and any of them may be NULL (not
 * copied).  Fails as gs_get_list_info does (no render yet, pairs dropped),
 * and with GS_ERR_INVALID_ARGUMENT after gs_render_noalloc, whose lists are
 * not kept.
 *   values        uint32 [K]: Gaussian indices; tile t's list is
 *                 values[offsets[t] .. offsets[t+1]), front to back, i.e.
 *                 all K pairs sorted by key (tile << 32 | depth bits), ties
 *                 by Gaussian index
 *   tile_offsets  uint32 [tiles+1], or NULL
 *   keys          uint64 [K], or NULL: key of each sorted pair, where depth
 *                 bits are the IEEE float32 bits of the camera-space depth */
gs_status gs_copy_lists(gs_context* ctx, uint32_t* values, uint32_t* tile_offsets, uint64_t* keys,
                        void* stream);

/* Projected Gaussians of the last render (any pointer may be NULL); after a
 * batched render every array holds n_views * n items, item v * n + i being
 * Gaussian i in view v.
 *   splats         float [n][12]: u_hi, v_hi, u_lo, v_lo, conic A, B, C,
 *                  opacity, r, g, b, depth, where the 2D centre is
 *                  u = u_hi + u_lo (float32 pair of the double value) and
 *                  the EWA falloff is exp(-0.5(A dx^2 + C dy^2) - B dx dy)
 *   depth_key      uint32 [n] float32 bits of the camera-space depth t_z
 *                  (the low half of every pair key of the Gaussian); every
 *                  Gaussian with a finite t_z has one, also when it is culled
 *                  or off screen and has no pair; 0xFFFFFFFF otherwise
 *   radius         int32 [n] 3-sigma radius in pixels, 0 if no tile
 *   tiles_touched  uint32 [n]
 *   rect           uint16 [n][4] tile rectangle x0, y0, x1, y1 (exclusive) */
gs_status gs_copy_projection(gs_context* ctx, float* splats, uint32_t* depth_key, int32_t* radius,
                             uint32_t* tiles_touched, uint16_t* rect, void* stream);

/* Tracing.  gs_set_profiling takes a set of GS_PROFILE_* flags (0 turns
 * tracing off) that apply to the following gs_render calls on ctx; an
 * unknown flag gives GS_ERR_INVALID_ARGUMENT.
 *
 * GS_PROFILE_STAGES: gs_render records HIP events on its stream between the
 * stages below; gs_get_stage_times synchronises on them and returns the
 * device time of each stage of the last render, in milliseconds, in this
 * order:
 *   0 project      (one kernel: cull, EWA projection, SH colour)
 *   1 depth_sort   (four LSD radix passes over the N depth keys)
 *   2 bin_row_count     (per-row counts of the depth-sorted Gaussians, row
 *                        offsets, chunk table of the second level)
 *   3 bin_row_scatter   (one kernel: per-row lists in depth order)
 *   4 bin_tile_count    (per-tile counts within each row, tile offsets)
 *   5 bin_tile_scatter  (one kernel: the sorted pair list)
 *   6 blend             (one kernel: per-tile compositing)
 * The host read of the pair count (pair_capacity 0) falls between stages 2
 * and 3 and belongs to neither.  count must be GS_NUM_STAGES; a last render
 * without this flag gives GS_ERR_INVALID_ARGUMENT.
 *
 * GS_PROFILE_BLEND_WORK: the blend runs a variant that counts its work
 * (a few extra instructions per evaluation and one atomic per wave, so it is
 * not the variant to time); gs_get_blend_stats returns, for the last render
 * (host array of 4, GS_ERR_INVALID_ARGUMENT if it was not counted):
 *   [0] (pixel, list entry) evaluations of Eq. 1's term, up to each pixel's
 *       termination -- the work the per-pixel walk of Sec. 4.5 requires
 *   [1] evaluations that passed the 1/255 alpha test and were composited
 *   [2] list entries staged from HBM into LDS (summed over tiles)
 *   [3] lane evaluations the kernel executed: 64 per (wave, staged entry)
 *       that the wave did not skip, whether or not its pixels needed it */
#define GS_NUM_STAGES 7
#define GS_PROFILE_STAGES 1
#define GS_PROFILE_BLEND_WORK 2

gs_status gs_set_profiling(gs_context* ctx, int32_t flags);

gs_status gs_get_stage_times(gs_context* ctx, float* ms, int32_t count);

gs_status gs_get_blend_stats(gs_context* ctx, uint64_t* stats4);

/* Per-tile blend trace of the last render counted with
 * GS_PROFILE_BLEND_WORK (host array [tiles][6], tiles = tiles_x * tiles_y of
 * that render, tile index ty * tiles_x + tx): [0] start and [1] end of the
 * tile's workgroup on the device's constant 100 MHz clock, [2] list entries
 * staged, [3] (wave, entry) bodies executed, [4] (pixel, entry) evaluations
 * up to each pixel's termination, [5] evaluations composited.  Per-tile work
 * and time are the GPU counterpart of the per-tile min/mean/max timings of
 * Table 2.  gs_get_blend_stats holds the sums over tiles.
 * GS_ERR_INVALID_ARGUMENT if the render was not counted or tiles differs. */
gs_status gs_get_blend_tile_work(gs_context* ctx, uint64_t* work, int64_t tiles);

/* Outcome of the last render's GS_RENDER_REUSE_ORDER attempt (host array of
 * 2, synchronises with that render): [0] 1 if the reused order held and the
 * radix sort was skipped, 0 if it ran; [1] the number of adjacent pairs of
 * the previous order that this frame's depths put out of order (the order's
 * churn between the two frames).  GS_ERR_INVALID_ARGUMENT if the last render
 * did not start from a previous order. */
gs_status gs_get_order_reuse(gs_context* ctx, uint32_t* out2);

/* Outcome of the last render's GS_RENDER_REUSE_LISTS comparison (host array
 * of 2, synchronises with that render or graph replay): [0] 1 if no
 * Gaussian's depth key or tile rectangle had changed and the previous lists
 * were kept (sort and binning skipped), else 0; [1] the number of (view,
 * Gaussian) items whose key or rectangle changed (each view's share
 * saturating at 2^32 - 1).  GS_ERR_INVALID_ARGUMENT if the last
 * render made no comparison (flag absent, or a render the flag is ignored
 * for). */
gs_status gs_get_list_reuse(gs_context* ctx, uint32_t* out2);

/* Launch shapes of the render, chosen per workload: the tile size (16, which
 * the keys of Sec. 3.1 and the lists depend on) is fixed, but how many items
 * a thread or wavefront carries in each stage, and how the blend's tiles are
 * dealt to the XCDs, change only speed.  Every supported value gives the same
 * image, final T, n_contrib, lists and projection, bit for bit.
 *   sort_items        keys per thread of a depth-sort block: 4, 8 or 16
 *   bin_row_items     depth-sorted Gaussians per lane of a row-binning
 *                     wavefront: 4, 8 or 16
 *   bin_tile_items    row entries per lane of a tile-binning wavefront:
 *                     8, 16 or 32
 *   blend_tile_group  consecutive tiles (row-major) dealt to one XCD by the
 *                     blend and its backward: 1 .. 64; or 0: every tile's
 *                     workgroup is dispatched heaviest first, by the work
 *                     (list entries walked) each tile took in the last
 *                     render on the context when it had the same tile
 *                     layout, else by list length -- the frame-to-frame
 *                     coherence of Sec. 5.7 applied to the load imbalance of
 *                     the per-tile blend (Sec. 6); or -1: the same order
 *                     as a work queue over the (view, tile) items of all
 *                     views, drained by a persistent grid of as many
 *                     workgroups as the device holds at once, each taking
 *                     the next item from an atomic head when it finishes
 *                     one; the backward follows its render's order
 *   blend_batch       list entries the blend stages from HBM into on-chip
 *                     memory per batch: 128, 256 or 512 (the backward
 *                     stages 256)
 * A new context starts at {8, 8, 16, 0, 256}.  gs_set_tuning applies to the
 * following renders and backwards (a backward uses its render's shapes; a
 * captured graph keeps those of its capture); GS_ERR_INVALID_ARGUMENT for an
 * unsupported value, leaving the tuning unchanged. */
typedef struct {
    int32_t sort_items;
    int32_t bin_row_items;
    int32_t bin_tile_items;
    int32_t blend_tile_group;
    int32_t blend_batch;
} gs_tuning;

gs_status gs_set_tuning(gs_context* ctx, const gs_tuning* tuning);
gs_status gs_get_tuning(gs_context* ctx, gs_tuning* out);

/* Autotuner: renders the given views (as gs_render_batched, whose outputs
 * it overwrites) with each candidate shape, one parameter at a time from the
 * context's current tuning -- sort_items scored by the depth-sort stage time,
 * bin_row_items and bin_tile_items by the four binning stages,
 * blend_tile_group and blend_batch by the blend -- each candidate once
 * untimed and then reps
 * times timed by the stage events, keeps the fastest value of each parameter
 * before tuning the next, and leaves the result as the context's tuning.
 *   out     the chosen tuning (may be NULL)
 *   out_ms  NULL, or host array [GS_TUNE_CANDIDATES]: the mean scored time
 *           of every candidate in the order sort_items 4, 8, 16;
 *           bin_row_items 4, 8, 16; bin_tile_items 8, 16, 32;
 *           blend_tile_group -1, 0, 1, 2, 4, 8, 16, 32, 64; blend_batch 128,
 *           256, 512
 * Profiling flags are restored afterwards.  Errors as gs_render_batched,
 * GS_ERR_INVALID_ARGUMENT for reps outside [1, 1000] or a context bound to a
 * graph; on error the tuning is left as it was. */
#define GS_TUNE_CANDIDATES 21
gs_status gs_autotune(gs_context* ctx, const gs_gaussians* g, const gs_view* views, int32_t n_views,
                      const gs_render_opts* opts, int32_t reps, void* stream, gs_tuning* out, float* out_ms);

#ifdef __cplusplus
}
#endif

#endif /* GSMI_H */
