// blend_stage.h -- staging of one list entry for the per-tile blend, shared
// by the forward (blend.hip) and backward (backward.hip) kernels so that both
// see the same per-entry values and take the same inclusion decisions.
#pragma once

#include "gs_internal.h"

namespace gsmi {

constexpr float kLog2e = 1.4426950408889634f;

// Smallest value of the quadratic form A x^2 + 2 B x y + C y^2 (positive
// definite) over the box [x0, x0 + 7] x [y0, y0 + 7] of pixel offsets, made a
// lower bound by subtracting 1e-5 of a bound on the size of its terms over
// the box (2 |B x y| <= |B| (x^2 + y^2)), which covers the float rounding of
// every evaluation.  The form is convex, so its minimum is 0 when the origin
// lies in the box and on an edge otherwise; on an edge it is a 1D quadratic
// minimised in closed form, at y = -(B / C) x or x = -(B / A) y (bc = B / C
// and ba = B / A, computed once per entry: the rounding of the minimiser
// moves the value by a term quadratic in that rounding, far inside the
// margin).
__device__ __forceinline__ float quad_min_over_box(float x0, float y0, float A, float B, float C, float bc, float ba)
{
    const float x1 = x0 + 7.0f, y1 = y0 + 7.0f;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return 0.0f;
    float q = INFINITY;
    const float xs[2] = {x0, x1}, ys[2] = {y0, y1};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float xe = xs[e];
        // clamp to [y0, y1] as one median-of-three (finite operands: the
        // same value as min(y1, max(y0, .)))
        const float y = __builtin_amdgcn_fmed3f(-bc * xe, y0, y1);
        q = fminf(q, A * xe * xe + 2.0f * B * xe * y + C * y * y);
        const float ye = ys[e];
        const float x = __builtin_amdgcn_fmed3f(-ba * ye, x0, x1);
        q = fminf(q, A * x * x + 2.0f * B * x * ye + C * ye * ye);
    }
    const float ab = fabsf(B);
    const float S = (A + ab) * fmaxf(x0 * x0, x1 * x1) + (C + ab) * fmaxf(y0 * y0, y1 * y1);
    return q - 1e-5f * (S + 1.0f);
}

// Stages one entry (its 48-byte record ra, rb, rc) for the tile with origin
// (ox, oy): v0 = centre - tile origin as a float hi/lo pair computed in double
// precision, v1 = conic scaled by -0.5 log2(e) (so alpha = opacity *
// exp2(A' dx^2 + B' dx dy + C' dy^2)) and opacity, v2 = colour and the list
// position.  Returns the 4-bit mask of the tile's 8x8 quads in which the entry
// can reach alpha 1/255 (a conservative bound: an entry outside it is skipped
// by every pixel of the quad).  v2.w holds the list position plus one (the
// n_contrib a pixel reports when this is its last composited entry).
__device__ __forceinline__ uint32_t stage_entry(const float4& ra, const float4& rb, const float4& rc, double ox,
                                                double oy, uint32_t pos, float4& v0, float4& v1, float4& v2)
{
    const double du = ((double)ra.x + (double)ra.z) - ox;
    const double dv = ((double)ra.y + (double)ra.w) - oy;
    const float du_hi = (float)du, dv_hi = (float)dv;
    uint32_t qmask = 0u;
    // the minimisers' slopes need no correct rounding (see quad_min_over_box):
    // a hardware reciprocal, not two divisions
    const float bc = rb.y * __builtin_amdgcn_rcpf(rb.z), ba = rb.y * __builtin_amdgcn_rcpf(rb.x);
    // opacity * exp(-q / 2) >= 1/255 where q <= 2 ln(255 opacity): one log
    // per entry instead of an exp per quad, with a margin (1e-4 of the
    // threshold's size) that covers the 1e-5 relative margin on alpha, the
    // fast log's error and the per-pixel exp2's, so no quad a pixel reaches
    // is dropped
    const float lt = 2.0f * __logf(255.0f * rb.w);
    const float thr = lt + 1e-4f * (1.0f + fabsf(lt));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float qmin = quad_min_over_box(du_hi - (float)((q & 1) * 8 + 7), dv_hi - (float)((q >> 1) * 8 + 7), rb.x,
                                             rb.y, rb.z, bc, ba);
        if (qmin <= thr) qmask |= 1u << q;
    }
    v0 = make_float4(du_hi, dv_hi, (float)(du - (double)du_hi), (float)(dv - (double)dv_hi));
    v1 = make_float4(-0.5f * kLog2e * rb.x, -kLog2e * rb.y, -0.5f * kLog2e * rb.z, rb.w);
    v2 = make_float4(rc.x, rc.y, rc.z, __int_as_float((int)(pos + 1u)));
    return qmask;
}

// Alpha of a staged entry (e0, e1) at the pixel with tile offset (fx, fy),
// shared by the forward and the backward so that both take the same
// decisions: the offset to the centre as (hi - pixel) + lo, then
// opacity * E with E = exp2(dx (A' dx + B' dy) + C' dy^2), clamped to 0.99.
// Returns alpha; dx, dy and the falloff E (for the backward) on the side.
__device__ __forceinline__ float entry_alpha(const float4& e0, const float4& e1, float fx, float fy, float& dx,
                                             float& dy, float& E)
{
    dx = (e0.x - fx) + e0.z;
    dy = (e0.y - fy) + e0.w;
    const float pw = fmaf(fmaf(e1.x, dx, e1.y * dy), dx, (e1.z * dy) * dy);
    E = __builtin_amdgcn_exp2f(pw);
    return fminf(0.99f, e1.w * E);
}

// Workgroup -> tile: tiles are cut into groups of `group` consecutive tiles
// (row-major), dealt to the 8 XCDs in turn (block b runs on XCD b % 8), so
// neighbouring tiles, which share list entries, share an XCD's L2.
__device__ __forceinline__ int blend_tile_of_block(int group)
{
    const int i = (int)(blockIdx.x >> 3);
    return ((i / group) * 8 + (int)(blockIdx.x & 7)) * group + i % group;
}

inline int blend_blocks(int64_t tiles, int group)
{
    return (int)(8 * group * ((tiles + 8 * group - 1) / (8 * group)));
}

// Workgroup -> tile when a dispatch order is given (heaviest tiles first,
// from the previous frame's per-tile work): block b takes order[b]; else the
// XCD groups above.
__device__ __forceinline__ int blend_tile(const uint32_t* order, int group)
{
    return order ? (int)order[blockIdx.x] : blend_tile_of_block(group);
}

inline int blend_grid(int64_t tiles, const uint32_t* order, int group)
{
    return order ? (int)tiles : blend_blocks(tiles, group);
}

}  // namespace gsmi
