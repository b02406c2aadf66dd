// blend.hip -- front-to-back alpha compositing per 16x16 screen tile (gfx950).
//
// Stage 4 of the render (Sec. 3.1) and the per-pixel walk of Sec. 4.5: every
// pixel accumulates Eq. 1 over its tile's depth-ordered list,
//   alpha_i = min(0.99, sigma_i * exp(-0.5 (A dx^2 + C dy^2) - B dx dy)),
// skipping alpha_i < 1/255 and stopping before the Gaussian that would take
// the transmittance below 1e-4 (early termination).
//
// One 256-lane workgroup (four wave64) owns one tile, one pixel per lane.
// Gaussians are staged through LDS in batches of 256: each lane gathers one
// 48-byte record, re-expresses the centre relative to the tile origin as a
// float hi/lo pair computed in double precision (so a pixel's dx, dy keep
// full float accuracy wherever the centre lies) and folds -0.5*log2(e) into
// the conic so the per-pixel work is one exp2 and a few FMAs.  Entries whose
// largest alpha over the whole tile is provably below 1/255 are dropped at
// staging (a conservative lower bound of the quadratic form over the tile's
// pixel box): every pixel would skip them, so the image is unchanged, and the
// 3-sigma square of the lists leaves many such (Gaussian, tile) pairs.  The
// same bound per 8x8 quad gives each entry a 4-bit mask: a wave owns one quad
// and steps over entries outside its reach with one scalar branch.  The
// per-pixel loop is predicated rather than branched; a wave leaves once all
// 64 of its pixels have terminated and the workgroup once all 256 have.  No
// MFMA: there is no dense contraction in this loop.
//
// Workgroup -> tile mapping is XCD-aware: the dispatcher deals consecutive
// workgroups round-robin to the 8 XCDs, so block b runs on XCD b % 8.  Tiles
// are cut into groups of a.group consecutive tiles (row-major; the autotuner
// picks the group size), dealt to the XCDs
// in turn: XCD x takes groups x, x + 8, x + 16, ... in screen order.  Each
// group's tiles share Gaussians in one L2, and every XCD gets an even share of
// every part of the screen: blend work per tile varies by an order of
// magnitude between the dense centre and sparse edges (tiles that never
// saturate walk their whole list), and contiguous bands per XCD would leave
// the XCDs with the heavy bands running long after the others finish.
#include "gs_internal.h"
#include "blend_stage.h"
#include "tile_order.h"

#include <atomic>

namespace gsmi {
namespace {

constexpr int kUnroll = 16;   // entries per unrolled group (a divisor of 64)
static_assert(64 % kUnroll == 0, "groups do not straddle a 64-entry mask word");
constexpr uint64_t kGroupMask = kUnroll == 64 ? ~0ull : ((1ull << kUnroll) - 1ull);

// Waves per SIMD the plain kernel asks for, by batch: 7 at 256 entries (at
// most 72 VGPRs; its batches wait on gathers and barriers, and more resident
// tiles hide more of that: 5 and 6 waves ran alike, 7 ran 4% faster, 8
// spilled and ran slower); 6 at 128, which spills at 7 (the half of the
// lanes that stage carries a predicate); 4 at 512, where each lane carries
// two entries' gathers (107 VGPRs).
template <int kBatch>
constexpr int blend_waves() { return kBatch == 256 ? 7 : (kBatch == 128 ? 6 : 4); }

// The LDS of one tile's walk (one instance per workgroup).
template <int kBatch>
struct BlendLds {
    float4 s0[kBatch + kUnroll];   // du_hi, dv_hi, du_lo, dv_lo  (centre - tile origin)
    float4 s1[kBatch + kUnroll];   // A', B', C', opacity  (A' = -0.5 log2(e) A, ...)
    float4 s2[kBatch + kUnroll];   // r, g, b, list position (int bits)
    uint32_t s_mask[kBatch + kUnroll];   // quads (waves) the entry can reach
    uint32_t s_wave_keep[4 * (kBatch > 256 ? kBatch / 256 : 1)];
    unsigned long long s_ev[4], s_co[4];   // tracing only
    uint32_t s_bodies[4];
};

// kStats: the tracing variant, which also records its work per tile
// (a.tile_work).  kBatch: list entries staged per batch (128, 256 or 512; an
// autotuner choice): each lane stages the entries tid, tid + 256 of the batch
// that exist, so 128 leaves half the lanes out of the staging.  The image
// does not depend on it; a smaller batch stages fewer entries past the point
// where every pixel has terminated, a larger one fewer barriers.  Called by
// all 256 threads of the workgroup with the same tile; the LDS is free again
// once every thread has returned.
template <bool kStats, int kBatch>
__device__ __forceinline__ void blend_tile_walk(const BlendArgs& a, uint64_t capacity, int tile, BlendLds<kBatch>& L)
{
    constexpr int kPer = kBatch > 256 ? kBatch / 256 : 1;   // entries a lane stages per batch
    constexpr int kWords = kBatch / 64;                     // 64-entry mask words of a batch
    static_assert(kBatch == 128 || kBatch == 256 || kBatch == 512, "batch of 128, 256 or 512 entries");
    float4* s0 = L.s0;
    float4* s1 = L.s1;
    float4* s2 = L.s2;
    uint32_t* s_mask = L.s_mask;
    uint32_t* s_wave_keep = L.s_wave_keep;
    if (tile >= a.tiles) return;
    // the view owning this global tile: its size, tile grid and outputs
    const ViewParams& vp = a.views[view_of_tile(a.views, a.n_views, (uint32_t)tile)];
    const int width = vp.width, height = vp.height;
    const int local = tile - (int)vp.tile_base;
    const int tx = local % vp.tiles_x, ty = local / vp.tiles_x;
    // the wave index is uniform: readfirstlane lets the compiler keep it scalar
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t t_start = kStats ? wall_clock64() : 0ull;
    // each wave owns one 8x8 quad of the tile
    const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const bool inside = px < width && py < height;
    uint64_t start = a.tile_offsets[tile], end = a.tile_offsets[tile + 1];
    if (end > capacity) end = capacity;
    if (start > end) start = end;
    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const float fx = (float)lx, fy = (float)ly;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    float Tr = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0, term = 0, composited = 0, staged = 0, bodies = 0;
    bool done = !inside;
    // software pipeline of the gathers: list values two batches ahead, the
    // 48-byte records one batch ahead, both overlapping the compositing.
    // Lane tid stages the batch entries tid + 256 p (p < kPer) below kBatch.
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t g_after[kPer];
    float4 na[kPer], nb[kPer], nc[kPer];
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
        const int slot = p * 256 + tid;
        const bool act = kBatch >= 256 || slot < kBatch;
        const uint32_t g_next = (act && start + slot < end) ? a.values[start + slot] : 0u;
        g_after[p] = (act && start + kBatch + slot < end) ? a.values[start + kBatch + slot] : 0u;
        na[p] = nb[p] = nc[p] = zero4;
        if (act && start + slot < end) {
            const float4* rec = reinterpret_cast<const float4*>(a.splats + g_next);
            na[p] = rec[0];
            nb[p] = rec[1];
            nc[p] = rec[2];
        }
    }
    uint64_t b0 = start;
    for (; b0 < end; b0 += kBatch) {
        if (__syncthreads_count(!done) == 0) break;
        // stage: the lane's entries, each dropped when no pixel of the tile
        // can reach alpha 1/255 (the per-pixel test would skip it everywhere)
        bool keep[kPer];
        uint32_t qmask[kPer];
        float4 v0[kPer], v1[kPer], v2[kPer];
#pragma unroll
        for (int p = 0; p < kPer; ++p) {
            const int slot = p * 256 + tid;
            const bool act = kBatch >= 256 || slot < kBatch;
            const float4 ra = na[p], rb = nb[p], rc = nc[p];
            if (act && b0 + kBatch + slot < end) {
                const float4* rec = reinterpret_cast<const float4*>(a.splats + g_after[p]);
                na[p] = rec[0];
                nb[p] = rec[1];
                nc[p] = rec[2];
            }
            g_after[p] = (act && b0 + 2 * kBatch + slot < end) ? a.values[b0 + 2 * kBatch + slot] : 0u;
            const uint64_t e = b0 + slot;
            keep[p] = false;
            qmask[p] = 0u;
            if (act && e < end) {
                qmask[p] = stage_entry(ra, rb, rc, ox, oy, (uint32_t)(e - start), v0[p], v1[p], v2[p]);
                keep[p] = qmask[p] != 0u;
            }
        }
        // order-preserving compaction of the kept entries: list order is
        // (p, wave, lane)
        uint64_t km[kPer];
#pragma unroll
        for (int p = 0; p < kPer; ++p) {
            km[p] = __ballot(keep[p]);
            if (lane == 0) s_wave_keep[p * 4 + wave] = (uint32_t)__popcll(km[p]);
        }
        if (kStats) staged += (end - b0 < (uint64_t)kBatch) ? (uint32_t)(end - b0) : (uint32_t)kBatch;
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kPer; ++p) {
            uint32_t slot = (uint32_t)__popcll(km[p] & lt);
            for (int i = 0; i < p * 4 + wave; ++i) slot += s_wave_keep[i];
            if (keep[p]) {
                s0[slot] = v0[p];
                s1[slot] = v1[p];
                s2[slot] = v2[p];
                s_mask[slot] = qmask[p];
            }
        }
        int nk = 0;
#pragma unroll
        for (int i = 0; i < 4 * kPer; ++i) nk += (int)s_wave_keep[i];
        if (tid < kUnroll) {   // padding entries reach no quad
            s0[nk + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
            s1[nk + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
            s2[nk + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
            s_mask[nk + tid] = 0u;
        }
        __syncthreads();
        // this wave's entries of the batch: bit j of bits[j / 64] when entry j
        // can reach the wave's quad (scalar registers, no per-entry LDS read)
        uint64_t bits[kWords];
#pragma unroll
        for (int q = 0; q < kWords; ++q) {
            const int jj = q * 64 + lane;
            bits[q] = __ballot(jj < nk && ((s_mask[jj] >> wave) & 1u));
        }
        for (int j0 = 0; j0 < nk; j0 += kUnroll) {
            if (__ballot(!done) == 0) break;   // whole wave finished
            const uint64_t word = bits[j0 >> 6] >> (j0 & 63);
            if ((word & kGroupMask) == 0) continue;   // none of the next kUnroll reaches the quad
            // the group's LDS byte offset in a VGPR: every entry below reads
            // at a constant offset from it (no per-entry address move)
            uint32_t gofs = (uint32_t)j0 * (uint32_t)sizeof(float4);
            __asm__ volatile("" : "+v"(gofs));
            const char* g0 = reinterpret_cast<const char*>(s0) + gofs;
            const char* g1 = reinterpret_cast<const char*>(s1) + gofs;
            const char* g2 = reinterpret_cast<const char*>(s2) + gofs;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                // an entry out of this quad's reach is skipped by the whole wave
                if (!((word >> u) & 1u)) continue;
                if (kStats) ++bodies;
                const float4 e0 = reinterpret_cast<const float4*>(g0)[u];
                const float4 e1 = reinterpret_cast<const float4*>(g1)[u];
                const float4 e2 = reinterpret_cast<const float4*>(g2)[u];
                float dx, dy, E;
                const float al = entry_alpha(e0, e1, fx, fy, dx, dy, E);
                const float tn = fmaf(-al, Tr, Tr);   // Tr (1 - al), rounded once
                const bool pass = al >= 1.0f / 255.0f;
                const bool stop = pass && tn < 1e-4f && !done;
                const bool take = pass && !stop && !done;
                const uint32_t pos1 = (uint32_t)__float_as_int(e2.w);   // list position + 1
                if (kStats) term = stop ? pos1 : term;
                done = done || stop;
                if (take) {   // under the lane mask: no selects
                    const float wt = al * Tr;
                    c0 = fmaf(wt, e2.x, c0);
                    c1 = fmaf(wt, e2.y, c1);
                    c2 = fmaf(wt, e2.z, c2);
                    Tr = tn;
                    last = pos1;
                }
                if (kStats) composited += take ? 1u : 0u;
            }
        }
    }
    if (kStats) {   // tracing only: one record per tile, no shared counters
        // a pixel examines its tile's list up to its terminating entry
        const uint32_t list_len = (uint32_t)(end - start);
        unsigned long long ev = inside ? (term ? term : list_len) : 0u, co = composited;
        for (int o = 32; o > 0; o >>= 1) {
            ev += __shfl_xor(ev, o, 64);
            co += __shfl_xor(co, o, 64);
        }
        if (lane == 0) {
            L.s_ev[wave] = ev;
            L.s_co[wave] = co;
            L.s_bodies[wave] = bodies;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long* w = a.tile_work + kTileWorkFields * (int64_t)tile;
            w[0] = t_start;
            w[1] = wall_clock64();
            w[2] = staged;
            w[3] = (unsigned long long)L.s_bodies[0] + L.s_bodies[1] + L.s_bodies[2] + L.s_bodies[3];
            w[4] = L.s_ev[0] + L.s_ev[1] + L.s_ev[2] + L.s_ev[3];
            w[5] = L.s_co[0] + L.s_co[1] + L.s_co[2] + L.s_co[3];
        }
    }
    // the work of this tile, for the next frame's dispatch order: list
    // entries walked before every pixel had terminated
    if (a.tile_cost && tid == 0) a.tile_cost[tile] = (uint32_t)((b0 < end ? b0 : end) - start);
    if (!inside) return;
    const int64_t P = (int64_t)width * height;
    const int64_t p = (int64_t)py * width + px;
    float* out_rgb = vp.out_rgb;
    out_rgb[p] = fmaf(Tr, a.bg[0], c0);
    out_rgb[P + p] = fmaf(Tr, a.bg[1], c1);
    out_rgb[2 * P + p] = fmaf(Tr, a.bg[2], c2);
    if (vp.out_T) vp.out_T[p] = Tr;
    if (vp.out_nc) vp.out_nc[p] = last;
}

// One workgroup per tile: workgroup b walks tile order[b] (heaviest first)
// or, without an order, the tile its XCD group assigns.  kStats keeps the
// compiler's own register budget, where the tracing counters need no spills.
template <bool kStats, int kBatch>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kStats ? 1 : blend_waves<kBatch>()))) void
blend_kernel(BlendArgs a, uint64_t capacity)
{
    __shared__ BlendLds<kBatch> lds;
    blend_tile_walk<kStats, kBatch>(a, capacity, blend_tile(a.order, a.group), lds);
}

// Persistent form: a grid of at most as many workgroups as the chip holds at
// once, each taking the next position of the heaviest-first order from an
// atomic head (a.queue, zero at the start of the frame) until the order is
// used up.  The work queue runs over the global tiles of every view, so the
// (view, tile) items of uneven cameras share one pool: a workgroup that
// finishes early takes the next heaviest item instead of idling while the
// dispatcher drains.  Every workgroup leaves once the head passes the tile
// count, so the grid always drains.  It asks for one wave per SIMD fewer
// than the plain kernel: the loop's own state spills at the plain count.
// Measured at 3M Gaussians / 1080p and on the 64-view batch it is slower
// than the dispatcher walking the same order one workgroup per tile
// (blend_group 0: 0.23 against 0.20 ms at 1080p), so the autotuner keeps it
// as a candidate only; claiming the next item before walking the current one
// needs a register across the walk and was slower still.
template <int kBatch>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(blend_waves<kBatch>() - 1))) void
blend_queue_kernel(BlendArgs a, uint64_t capacity)
{
    __shared__ BlendLds<kBatch> lds;
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();   // every thread has read s_item before thread 0 writes the next
        if ((int64_t)item >= a.tiles) break;
        blend_tile_walk<false, kBatch>(a, capacity, (int)a.order[item], lds);
    }
}

// The order of a layout's first frame (by list length; later frames take the
// previous frame's walked entries, ordered beside the projection): one
// 1024-thread workgroup, each tile's bucket kept in LDS between the passes.
constexpr int kOrderThreads = 1024;
constexpr int kOrderKeptTiles = 32768;
__global__ __launch_bounds__(kOrderThreads) void blend_order_kernel(const uint32_t* __restrict__ cost,
                                                                    const uint32_t* __restrict__ offsets,
                                                                    int64_t tiles, uint32_t* __restrict__ order)
{
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint16_t s_bucket[kOrderKeptTiles];
    __shared__ uint32_t wsum[kOrderThreads / 64];
    order_heaviest_first<kOrderThreads>(cost, offsets, tiles, order, hist, wsum, s_bucket, kOrderKeptTiles);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// keys[j] = tile << 32 | depth bits of values[j], one block per tile
__global__ __launch_bounds__(256) void write_keys_kernel(const uint32_t* __restrict__ values,
                                                         const uint32_t* __restrict__ offsets,
                                                         const uint32_t* __restrict__ depth_key,
                                                         uint64_t* __restrict__ keys)
{
    const uint64_t t = blockIdx.x;
    const uint32_t s = offsets[t], e = offsets[t + 1];
    for (uint32_t j = s + threadIdx.x; j < e; j += 256) keys[j] = (t << 32) | depth_key[values[j]];
}

// Workgroups of a 256-thread kernel that the current device holds at once
// (resident per compute unit times compute units), cached per device and
// batch (contexts on several host threads may fill the cache at once: each
// writes the same value); 0 when the runtime cannot say.
template <typename K>
int64_t resident_blocks(K kernel, int batch)
{
    constexpr int kDevices = 64;
    static std::atomic<int64_t> cache[kDevices][3];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return 0;
    const int slot = batch == 128 ? 0 : (batch == 256 ? 1 : 2);
    const int64_t known = cache[dev][slot].load(std::memory_order_relaxed);
    if (known > 0) return known;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
        cus <= 0)
        return 0;
    const int64_t blocks = (int64_t)per_cu * cus;
    cache[dev][slot].store(blocks, std::memory_order_relaxed);
    return blocks;
}

}  // namespace

hipError_t launch_blend(const BlendArgs& a, uint64_t capacity, hipStream_t s)
{
    const int64_t T = a.tiles;
    if (T <= 0) return hipSuccess;
    if (a.queue && a.order && !a.tile_work) {   // persistent grid over the heaviest-first queue
        auto go = [&](auto kernel) {
            const int64_t r = resident_blocks(kernel, a.batch);   // 0: one workgroup per tile
            const int blocks = (int)(r > 0 ? std::min<int64_t>(T, r) : T);
            hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, a, capacity);
        };
        switch (a.batch) {
        case 128: go(blend_queue_kernel<128>); break;
        case 512: go(blend_queue_kernel<512>); break;
        case 256: go(blend_queue_kernel<256>); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int blocks = blend_grid(T, a.order, a.group);
    auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, a, capacity); };
    switch (a.batch) {
    case 128: a.tile_work ? go(blend_kernel<true, 128>) : go(blend_kernel<false, 128>); break;
    case 512: a.tile_work ? go(blend_kernel<true, 512>) : go(blend_kernel<false, 512>); break;
    case 256: a.tile_work ? go(blend_kernel<true, 256>) : go(blend_kernel<false, 256>); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blend_order(const uint32_t* cost, const uint32_t* tile_offsets, int64_t tiles, uint32_t* order,
                              hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(blend_order_kernel, dim3(1), dim3(kOrderThreads), 0, s, cost, tile_offsets, tiles, order);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_write_keys(const uint32_t* values, const uint32_t* tile_offsets, const uint32_t* depth_key,
                             int64_t tiles, uint64_t* keys, hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(write_keys_kernel, dim3((unsigned)tiles), dim3(256), 0, s, values, tile_offsets, depth_key,
                       keys);
    return hipGetLastError();
}

}  // namespace gsmi
