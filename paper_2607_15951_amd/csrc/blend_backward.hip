// blend_backward.hip -- gradient of the per-tile front-to-back blend.
//
// The forward of Eq. 1 gives, per pixel, C = sum_j a_j T_j c_j + T_f bg with
// T_j = prod_{i<j} (1 - a_i) over the composited entries.  For a loss L with
// G = dL/dC and G_T = dL/dT_f, an entry j that the pixel composited gets
//   dL/dc_j = G a_j T_j
//   dL/da_j = G . (T_j c_j - (S_j + T_f bg) / (1 - a_j)) - G_T T_f / (1 - a_j)
// where S_j = sum_{k>j} a_k T_k c_k is the colour composited after j.  The
// pass is recomputed rather than stored: walking the list front to back with
// the forward's own arithmetic gives the same a_j and T_j, S_j is the
// forward's colour minus the running sum, and the walk stops at the pixel's
// n_contrib (one past its last composited entry).  Through a = min(0.99,
// opacity exp(p)) with p = -0.5 (A dx^2 + C dy^2) - B dx dy the gradient
// reaches the opacity, the conic and the centre; a clamped alpha passes none.
//
// Layout as the forward: one workgroup of four waves per 16x16 tile, one pixel
// per lane, entries staged through LDS with the same per-quad reach masks.
// Per entry, each wave sums its 64 pixels' nine gradients (a transposed
// butterfly, below) and adds them into an LDS row of the staged entry; after
// the batch every row with a contribution goes to HBM with nine atomic adds
// (once per tile and entry).
#include "blend_stage.h"

namespace gsmi {
namespace {

constexpr float kLn2 = 0.69314718055994531f;

// The value of the lane whose index differs in bit kBit: DPP quad
// permutations for bits 0 and 1, ds_swizzle (bit-mask mode, within 32 lanes)
// for bits 2 to 4, ds_bpermute across the two halves for bit 5.
template <int kBit>
__device__ __forceinline__ float lane_xor(float v)
{
    const int x = __float_as_int(v);
    if constexpr (kBit == 0) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
    else if constexpr (kBit == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
    else if constexpr (kBit < 5) return __int_as_float(__builtin_amdgcn_ds_swizzle(x, 0x1F | ((1 << kBit) << 10)));
    else return __shfl_xor(v, 32, 64);
}

// One butterfly step over lane bit kBit for pairs (lo, hi): a lane whose bit
// is clear keeps lo plus its partner's lo, the other keeps hi plus its
// partner's hi, so one move per pair halves the values each lane carries.
template <int kBit>
__device__ __forceinline__ float trade(float lo, float hi, bool upper)
{
    return (upper ? hi : lo) + lane_xor<kBit>(upper ? lo : hi);
}

// Wave sums of the nine values g[0..8] of every lane, with 13 cross-lane moves
// instead of 9 x 6: four trading steps over lane bits 0-3 leave each lane one
// value summed over its 16-lane row, two plain steps over bits 4-5 finish the
// sum.  Returns the sum a lane holds and sets slot to the index of its value,
// or to -1 for a padding slot; lanes 0-15 hold each of the nine sums once.
__device__ __forceinline__ float wave_sum9(const float g[kGrad2d], int lane, int& slot)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
    float a[6], c[4], d[2];
#pragma unroll
    for (int i = 0; i < 5; ++i) a[i] = trade<0>(g[i], i < 4 ? g[5 + i] : 0.0f, b0);   // g0-4 | g5-8, 0
    a[5] = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = trade<1>(a[i], a[3 + i], b1);
    c[3] = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i) d[i] = trade<2>(c[i], c[2 + i], b2);
    float e = trade<3>(d[0], d[1], b3);
    e += lane_xor<4>(e);
    e += lane_xor<5>(e);
    const int ic = (b2 ? 2 : 0) + (b3 ? 1 : 0);    // index into c
    const int real = b1 ? (b0 ? 1 : 2) : 3;         // c entries that hold a value
    slot = (lane < 16 && ic < real) ? (b0 ? 5 : 0) + (b1 ? 3 : 0) + ic : -1;
    return e;
}

// 6 waves per SIMD (79 VGPRs, no spills; the compiler's own budget of 84
// leaves 5): its 23.8 KB of LDS also allows 6 tiles per CU
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void blend_backward_kernel(
    BlendBackArgs a, uint64_t capacity)
{
    __shared__ float4 s0[256];   // du_hi, dv_hi, du_lo, dv_lo
    __shared__ float4 s1[256];   // A', B', C', opacity
    __shared__ float4 s2[256];   // r, g, b, list position
    __shared__ uint32_t s_mask[256];
    __shared__ uint32_t s_item[256];
    __shared__ float s_acc[256][kGrad2d];
    __shared__ uint32_t s_wave_keep[4];
    const int tile = blend_tile(a.order, a.group);
    if (tile >= a.tiles) return;
    const ViewParams& vp = a.views[view_of_tile(a.views, a.n_views, (uint32_t)tile)];
    const int width = vp.width, height = vp.height;
    const int local = tile - (int)vp.tile_base;
    const int tx = local % vp.tiles_x, ty = local / vp.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const bool inside = px < width && py < height;
    uint64_t start = a.tile_offsets[tile], end = a.tile_offsets[tile + 1];
    if (end > capacity) end = capacity;
    if (start > end) start = end;
    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const float fx = (float)lx, fy = (float)ly;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // the pixel's forward outputs and loss gradients
    float G0 = 0.f, G1 = 0.f, G2 = 0.f, GT = 0.f, Tf = 1.f, S0 = 0.f, S1 = 0.f, S2 = 0.f;
    uint32_t nc = 0;
    if (inside) {
        const int64_t P = (int64_t)width * height, p = (int64_t)py * width + px;
        G0 = vp.grad_rgb[p];
        G1 = vp.grad_rgb[P + p];
        G2 = vp.grad_rgb[2 * P + p];
        GT = vp.grad_T ? vp.grad_T[p] : 0.f;
        Tf = vp.out_T[p];
        nc = vp.out_nc[p];
        // colour composited over the whole list, without the background
        S0 = vp.out_rgb[p] - Tf * a.bg[0];
        S1 = vp.out_rgb[P + p] - Tf * a.bg[1];
        S2 = vp.out_rgb[2 * P + p] - Tf * a.bg[2];
    }
    // the part of dL/da_j that does not depend on j's colour: background and
    // the final transmittance (both scale with T_f / (1 - a_j))
    const float Gbg = G0 * a.bg[0] + G1 * a.bg[1] + G2 * a.bg[2] + GT;
    float Tr = 1.0f;
    bool done = !inside || nc == 0;

    for (uint64_t b0 = start; b0 < end; b0 += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const uint64_t e = b0 + tid;
        bool keep = false;
        uint32_t qmask = 0u, item = 0u;
        float4 v0, v1, v2;
        if (e < end) {
            item = a.values[e];
            const float4* rec = reinterpret_cast<const float4*>(a.splats + item);
            qmask = stage_entry(rec[0], rec[1], rec[2], ox, oy, (uint32_t)(e - start), v0, v1, v2);
            keep = qmask != 0u;
        }
        const uint64_t km = __ballot(keep);
        if (lane == 0) s_wave_keep[wave] = (uint32_t)__popcll(km);
        __syncthreads();
        uint32_t slot = (uint32_t)__popcll(km & lt);
        for (int w = 0; w < wave; ++w) slot += s_wave_keep[w];
        const int nk = (int)(s_wave_keep[0] + s_wave_keep[1] + s_wave_keep[2] + s_wave_keep[3]);
        if (keep) {
            s0[slot] = v0;
            s1[slot] = v1;
            s2[slot] = v2;
            s_mask[slot] = qmask;
            s_item[slot] = item;
        }
        for (int k = tid; k < 256 * kGrad2d; k += 256) (&s_acc[0][0])[k] = 0.f;
        __syncthreads();
        uint64_t bits[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = q * 64 + lane;
            bits[q] = __ballot(jj < nk && ((s_mask[jj] >> wave) & 1u));
        }
        for (int j = 0; j < nk; ++j) {
            if (!((bits[j >> 6] >> (j & 63)) & 1u)) continue;
            if (__ballot(!done) == 0) break;   // every pixel of the wave is past its last entry
            const float4 e0 = s0[j], e1 = s1[j], e2 = s2[j];
            const uint32_t pos1 = (uint32_t)__float_as_int(e2.w);   // list position + 1
            if (!done && pos1 > nc) done = true;                      // past the pixel's last entry
            float dx, dy, E;
            const float al = entry_alpha(e0, e1, fx, fy, dx, dy, E);
            const float araw = e1.w * E;
            const bool take = !done && al >= 1.0f / 255.0f;
            float g[kGrad2d];
#pragma unroll
            for (int k = 0; k < kGrad2d; ++k) g[k] = 0.f;
            if (take) {
                const float w = al * Tr;
                S0 -= w * e2.x;   // colour composited after this entry
                S1 -= w * e2.y;
                S2 -= w * e2.z;
                g[6] = G0 * w;
                g[7] = G1 * w;
                g[8] = G2 * w;
                const float inv = __builtin_amdgcn_rcpf(1.0f - al);   // 1 - al >= 0.01
                const float ga = (G0 * e2.x + G1 * e2.y + G2 * e2.z) * Tr -
                                 (G0 * S0 + G1 * S1 + G2 * S2 + Gbg * Tf) * inv;
                if (araw <= 0.99f) {
                    const float gp = ga * al;   // dL/dp, p the exponent of exp
                    g[5] = ga * E;
                    g[2] = -0.5f * dx * dx * gp;
                    g[3] = -dx * dy * gp;
                    g[4] = -0.5f * dy * dy * gp;
                    // dp/d(dx) = -(A dx + B dy) = ln2 (2 A' dx + B' dy)
                    g[0] = gp * kLn2 * (2.0f * e1.x * dx + e1.y * dy);
                    g[1] = gp * kLn2 * (2.0f * e1.z * dy + e1.y * dx);
                }
                Tr = fmaf(-al, Tr, Tr);   // as the forward: Tr (1 - al), rounded once
            }
            if (__ballot(take) != 0) {
                int slot;
                const float v = wave_sum9(g, lane, slot);
                if (slot >= 0) atomicAdd(&s_acc[j][slot], v);
            }
        }
        __syncthreads();
        // one set of atomic adds per staged entry and tile
        for (int k = tid; k < nk * kGrad2d; k += 256) {
            const int j = k / kGrad2d, c = k % kGrad2d;
            const float v = s_acc[j][c];
            if (v != 0.f) unsafeAtomicAdd(&a.grad2d[(int64_t)s_item[j] * kGrad2d + c], v);
        }
    }
}

}  // namespace

hipError_t launch_blend_backward(const BlendBackArgs& a, uint64_t capacity, hipStream_t s)
{
    if (a.tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(blend_backward_kernel, dim3(blend_grid(a.tiles, a.order, a.group)), dim3(256), 0, s, a, capacity);
    return hipGetLastError();
}

}  // namespace gsmi
