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
// the conic so the per-pixel work is one exp2 and a few FMAs.  The workgroup
// leaves as soon as every pixel has terminated (a barrier count of the lanes
// still running).  No MFMA: there is no dense contraction in this loop.
//
// Workgroup -> tile mapping is XCD-aware: the dispatcher deals consecutive
// workgroups round-robin to the 8 XCDs, so block b takes tile
// (b % 8) * ceil(T/8) + b / 8 and each XCD's L2 serves a contiguous band of
// tiles whose lists share Gaussians.
#include "gs_internal.h"

namespace gsmi {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

__global__ __launch_bounds__(256) void blend_kernel(BlendArgs a, uint64_t capacity)
{
    __shared__ float4 s0[256];   // du_hi, dv_hi, du_lo, dv_lo  (centre - tile origin)
    __shared__ float4 s1[256];   // A', B', C', opacity         (A' = -0.5 log2(e) A, ...)
    __shared__ float4 s2[256];   // r, g, b, -
    const int T = a.tiles_x * a.tiles_y;
    const int per_xcd = (T + 7) / 8;
    const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= T) return;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int tid = threadIdx.x;
    const int lx = tid & 15, ly = tid >> 4;
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const bool inside = px < a.width && py < a.height;
    uint64_t start = a.tile_offsets[tile], end = a.tile_offsets[tile + 1];
    if (end > capacity) end = capacity;
    if (start > end) start = end;
    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const float fx = (float)lx, fy = (float)ly;

    float Tr = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0, examined = 0, composited = 0, staged = 0;
    bool done = !inside;
    for (uint64_t b0 = start; b0 < end; b0 += 256) {
        if (__syncthreads_count(!done) == 0) break;
        staged += (end - b0 < 256) ? (uint32_t)(end - b0) : 256u;
        const uint64_t e = b0 + tid;
        if (e < end) {
            const uint32_t g = a.values[e];
            const float4* rec = reinterpret_cast<const float4*>(a.splats + g);
            const float4 ra = rec[0], rb = rec[1], rc = rec[2];
            // centre relative to the tile origin as a float pair: the per-pixel
            // offset (hi - lx) + lo then carries ~2 ulp of its own size
            const double du = ((double)ra.x + (double)ra.z) - ox;
            const double dv = ((double)ra.y + (double)ra.w) - oy;
            const float du_hi = (float)du, dv_hi = (float)dv;
            s0[tid] = make_float4(du_hi, dv_hi, (float)(du - (double)du_hi), (float)(dv - (double)dv_hi));
            s1[tid] = make_float4(-0.5f * kLog2e * rb.x, -kLog2e * rb.y, -0.5f * kLog2e * rb.z, rb.w);
            s2[tid] = rc;
        }
        __syncthreads();
        if (!done) {
            const int cnt = (end - b0 < 256) ? (int)(end - b0) : 256;
            int j = 0;
            for (; j < cnt; ++j) {
                const float4 e0 = s0[j];
                const float4 e1 = s1[j];
                const float dx = (e0.x - fx) + e0.z;
                const float dy = (e0.y - fy) + e0.w;
                const float pw = fmaf(e1.x * dx, dx, fmaf(e1.z * dy, dy, (e1.y * dx) * dy));
                const float al = fminf(0.99f, e1.w * __builtin_amdgcn_exp2f(pw));
                if (al < 1.0f / 255.0f) continue;
                const float tn = Tr * (1.0f - al);
                if (tn < 1e-4f) {
                    done = true;
                    break;
                }
                ++composited;
                const float4 e2 = s2[j];
                const float wgt = al * Tr;
                c0 = fmaf(wgt, e2.x, c0);
                c1 = fmaf(wgt, e2.y, c1);
                c2 = fmaf(wgt, e2.z, c2);
                Tr = tn;
                last = (uint32_t)(b0 - start) + (uint32_t)j + 1u;
            }
            examined += (uint32_t)(j < cnt ? j + 1 : cnt);
        }
    }
    if (a.stats) {   // tracing only: one atomic per wave
        unsigned long long ev = examined, co = composited;
        for (int o = 32; o > 0; o >>= 1) {
            ev += __shfl_xor(ev, o, 64);
            co += __shfl_xor(co, o, 64);
        }
        if ((tid & 63) == 0) {
            atomicAdd(&a.stats[0], ev);
            atomicAdd(&a.stats[1], co);
        }
        if (tid == 0) atomicAdd(&a.stats[2], (unsigned long long)staged);
    }
    if (!inside) return;
    const int64_t P = (int64_t)a.width * a.height;
    const int64_t p = (int64_t)py * a.width + px;
    a.out_rgb[p] = fmaf(Tr, a.bg[0], c0);
    a.out_rgb[P + p] = fmaf(Tr, a.bg[1], c1);
    a.out_rgb[2 * P + p] = fmaf(Tr, a.bg[2], c2);
    if (a.out_T) a.out_T[p] = Tr;
    if (a.out_nc) a.out_nc[p] = last;
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

}  // namespace

hipError_t launch_blend(const BlendArgs& a, uint64_t capacity, hipStream_t s)
{
    const int T = a.tiles_x * a.tiles_y;
    const int blocks = 8 * ((T + 7) / 8);
    hipLaunchKernelGGL(blend_kernel, dim3(blocks), dim3(256), 0, s, a, capacity);
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
