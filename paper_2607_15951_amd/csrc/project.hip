// project.hip -- per-Gaussian cull + EWA projection + SH colour (gfx950).
//
// Stages 1-2 of the four-stage render (Sec. 3.1): frustum (near-plane) cull,
// projection to a 2D centre and conic, the 3-sigma square bound of Sec. 4.4,
// opacity sigma(alpha) of Eq. 1 and view-dependent SH colour.  One lane per
// Gaussian; structure-of-arrays inputs make every load a coalesced stream.
//
// Precision.  The geometry that decides integers -- culling, the bounding
// radius, the tile rectangle -- and the sort key's depth are evaluated in IEEE
// double precision in a fixed operation order with FMA contraction disabled,
// so that they are reproducible bit for bit on any IEEE machine that follows
// the same order.  On gfx950 the FP64 vector rate is half the FP32 rate and
// this kernel is bound by HBM reads (up to 236 B per Gaussian), so the double
// arithmetic costs no frame time.  Colour and opacity are FP32.
#include "gs_internal.h"
#include "tile_order.h"

#include <hip/hip_fp16.h>

namespace gsmi {
namespace {

template <int DT>
__device__ __forceinline__ float load_attr(const void* p, int64_t idx)
{
    if constexpr (DT == 0) {
        return static_cast<const float*>(p)[idx];
    } else if constexpr (DT == 1) {
        uint32_t b = static_cast<const uint16_t*>(p)[idx];
        return __uint_as_float(b << 16);
    } else {
        return __half2float(static_cast<const __half*>(p)[idx]);
    }
}

// Real SH basis to degree 3 in Cartesian form (unit direction x, y, z), index
// k = l*l + l + m; the sign convention carries the Condon-Shortley phase.
__device__ __forceinline__ void sh_basis(float x, float y, float z, int degree, float Y[16])
{
    Y[0] = 0.28209479177387814f;
    if (degree < 1) return;
    const float c1 = 0.48860251190291992f;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    Y[4] = 1.0925484305920792f * xy;
    Y[5] = -1.0925484305920792f * yz;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * xz;
    Y[8] = 0.54627421529603959f * (xx - yy);
    if (degree < 3) return;
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    Y[10] = 2.8906114426405538f * xy * z;
    Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

struct Geometry {
    double tz, u, v;
    double A, B, C;
    int32_t radius;
};

}  // namespace

size_t project_partials_elems(int64_t n, int n_views)
{
    return (size_t)(4 * ((n + 255) / 256 + 1) * (size_t)(n_views > 0 ? n_views : 1));
}

namespace {

// World-space covariance Sg = (Q S)(Q S)^T of a Gaussian (rotation Q of the
// normalised quaternion, S = diag(exp(log_scale))), in double precision with
// the operation order written here.  False for a zero or non-finite
// quaternion (the Gaussian is culled in every view).
__device__ __forceinline__ bool world_covariance(double l0, double l1, double l2, double qw, double qx, double qy,
                                                 double qz, double Sg[9])
{
#pragma clang fp contract(off)
    const double n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(n2 > 0.0) || !isfinite(n2)) return false;
    const double qn = sqrt(n2);
    const double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    // rotation matrix of the unit quaternion, row-major
    double Q[9];
    Q[0] = 1.0 - 2.0 * (y * y + z * z);
    Q[1] = 2.0 * (x * y - w * z);
    Q[2] = 2.0 * (x * z + w * y);
    Q[3] = 2.0 * (x * y + w * z);
    Q[4] = 1.0 - 2.0 * (x * x + z * z);
    Q[5] = 2.0 * (y * z - w * x);
    Q[6] = 2.0 * (x * z - w * y);
    Q[7] = 2.0 * (y * z + w * x);
    Q[8] = 1.0 - 2.0 * (x * x + y * y);

    // M = Q diag(exp(s)); world covariance Sg = M M^T
    const double s0 = exp(l0), s1 = exp(l1), s2 = exp(l2);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = Q[3 * r + 0] * s0;
        M[3 * r + 1] = Q[3 * r + 1] * s1;
        M[3 * r + 2] = Q[3 * r + 2] * s2;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Sg[3 * r + c] = (M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1]) + M[3 * r + 2] * M[3 * c + 2];
    return true;
}

// Culling and projection of one Gaussian (centre m, world covariance Sg) in
// one view, in double precision.  Returns false for a culled Gaussian.  The
// expression shapes below fix the rounding order.
__device__ __forceinline__ bool project_view(const ViewParams& vp, double mx, double my, double mz,
                                             const double Sg[9], Geometry& g)
{
#pragma clang fp contract(off)
    const double* W = vp.R;
    const double tx = ((W[0] * mx + W[1] * my) + W[2] * mz) + vp.t[0];
    const double ty = ((W[3] * mx + W[4] * my) + W[5] * mz) + vp.t[1];
    const double tz = ((W[6] * mx + W[7] * my) + W[8] * mz) + vp.t[2];
    if (!(tz > vp.near_plane) || !isfinite(tx) || !isfinite(ty) || !isfinite(tz)) return false;

    // camera-space covariance V = W Sg W^T (left product first)
    double L[9], V[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            L[3 * r + c] = (W[3 * r] * Sg[c] + W[3 * r + 1] * Sg[3 + c]) + W[3 * r + 2] * Sg[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            V[3 * r + c] = (L[3 * r] * W[3 * c] + L[3 * r + 1] * W[3 * c + 1]) + L[3 * r + 2] * W[3 * c + 2];

    // perspective Jacobian with x/z, y/z clamped to 1.3x the half-image tangent
    const double limx = 1.3 * ((0.5 * (double)vp.width) / vp.fx);
    const double limy = 1.3 * ((0.5 * (double)vp.height) / vp.fy);
    const double xcl = fmin(limx, fmax(-limx, tx / tz)) * tz;
    const double ycl = fmin(limy, fmax(-limy, ty / tz)) * tz;
    double Jm[6];
    Jm[0] = vp.fx / tz;
    Jm[1] = 0.0;
    Jm[2] = -(vp.fx * xcl) / (tz * tz);
    Jm[3] = 0.0;
    Jm[4] = vp.fy / tz;
    Jm[5] = -(vp.fy * ycl) / (tz * tz);
    double Bm[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Bm[3 * r + c] = (Jm[3 * r] * V[c] + Jm[3 * r + 1] * V[3 + c]) + Jm[3 * r + 2] * V[6 + c];
    const double p00 = (Bm[0] * Jm[0] + Bm[1] * Jm[1]) + Bm[2] * Jm[2];
    const double p01 = (Bm[0] * Jm[3] + Bm[1] * Jm[4]) + Bm[2] * Jm[5];
    const double p11 = (Bm[3] * Jm[3] + Bm[4] * Jm[4]) + Bm[5] * Jm[5];

    // EWA low-pass of 0.3 px^2, then the conic (inverse 2D covariance)
    const double ca = p00 + 0.3, cb = p01, cc = p11 + 0.3;
    const double det = ca * cc - cb * cb;
    if (!(det > 0.0) || !isfinite(det)) return false;
    g.A = cc / det;
    g.B = -cb / det;
    g.C = ca / det;

    // 3 sigma of the larger eigenvalue, whole pixels
    const double mid = 0.5 * (ca + cc);
    const double lam = mid + sqrt(fmax(0.0, mid * mid - det));
    const double r = ceil(3.0 * sqrt(lam));
    if (!(r > 0.0) || !(r < 1e9)) return false;
    g.radius = (int32_t)r;

    g.u = (vp.fx * tx) / tz + vp.cx;
    g.v = (vp.fy * ty) / tz + vp.cy;
    if (!isfinite(g.u) || !isfinite(g.v)) return false;
    g.tz = tz;
    return true;
}

// kOneView: the single-image render (one view, no loop-carried state, so the
// compiler schedules it as straight-line code)
template <int DT, int DEG, bool kOneView>
__global__ __launch_bounds__(256) void project_kernel(ProjectArgs a)
{
    constexpr int ncoef = (DEG + 1) * (DEG + 1);
    // the blend's dispatch order, when asked for, is workgroup 0's work: it
    // needs only the previous frame's per-tile costs, so it runs beside the
    // projection; the Gaussians go to workgroups 1 and up
    int64_t blk = blockIdx.x;
    if (a.order) {
        if (blockIdx.x == 0) {
            __shared__ uint32_t s_hist[kOrderBuckets], s_wsum[4];
            order_heaviest_first<256>(a.order_cost, nullptr, a.order_tiles, a.order, s_hist, s_wsum, nullptr, 0);
            return;
        }
        blk -= 1;
    }
    // lanes past n stay active (reading Gaussian 0) until the wave reduction
    const int64_t i_raw = blk * 256 + threadIdx.x;
    const bool valid = i_raw < a.n;
    const int64_t i = valid ? i_raw : 0;
    const int64_t n = a.n;
    // every attribute load is issued before any arithmetic, so a wave has all
    // of its 11 + 3 (DEG+1)^2 coalesced streams in flight at once
    const float mxf = a.means[i], myf = a.means[n + i], mzf = a.means[2 * n + i];
    const float l0 = load_attr<DT>(a.log_scales, i);
    const float l1 = load_attr<DT>(a.log_scales, n + i);
    const float l2 = load_attr<DT>(a.log_scales, 2 * n + i);
    const float qw = load_attr<DT>(a.quats, i);
    const float qx = load_attr<DT>(a.quats, n + i);
    const float qy = load_attr<DT>(a.quats, 2 * n + i);
    const float qz = load_attr<DT>(a.quats, 3 * n + i);
    const float logit = load_attr<DT>(a.logits, i);
    float coef[3 * ncoef];
#pragma unroll
    for (int k = 0; k < 3 * ncoef; ++k) coef[k] = load_attr<DT>(a.sh, (int64_t)k * n + i);

    double Sg[9];
    const bool cov_ok = world_covariance(l0, l1, l2, qw, qx, qy, qz, Sg);
    // sigmoid in double, rounded once: the opacity carries one float rounding
    // whatever the logit (a float exp of -logit would carry about |logit| of them)
    const float opacity = (float)(1.0 / (1.0 + exp(-(double)logit)));
    __shared__ uint32_t s_vis[4], s_pairs[4], s_front[4], s_changed[4];

    const int n_views = kOneView ? 1 : a.n_views;
    for (int v = 0; v < n_views; ++v) {
        const ViewParams& vp = a.views[v];
        Geometry g;
        const bool ok = cov_ok && project_view(vp, mxf, myf, mzf, Sg, g);
        // the depth key: every Gaussian with a finite depth keeps one, on
        // screen or not, culled or not (an off-screen or culled Gaussian
        // yields no pair), so the depth order changes little between nearby
        // frames even where Gaussians cross the screen edge or the near plane
        // (see launch_order_reuse); t_z as project_view computes it
        const double tz_key = ((vp.R[6] * (double)mxf + vp.R[7] * (double)myf) + vp.R[8] * (double)mzf) + vp.t[2];
        const bool keyed = isfinite(tz_key);

        uint32_t tiles = 0;
        ushort4 rc = make_ushort4(0, 0, 0, 0);
        if (ok && valid) {
            const double big = 1073741824.0;
            const double uc = fmin(big, fmax(-big, g.u)), vc = fmin(big, fmax(-big, g.v));
            int64_t xlo = (int64_t)ceil(uc) - g.radius, xhi = (int64_t)floor(uc) + g.radius;
            int64_t ylo = (int64_t)ceil(vc) - g.radius, yhi = (int64_t)floor(vc) + g.radius;
            if (!(xhi < 0 || xlo > vp.width - 1 || yhi < 0 || ylo > vp.height - 1)) {
                xlo = xlo < 0 ? 0 : xlo;
                ylo = ylo < 0 ? 0 : ylo;
                xhi = xhi > vp.width - 1 ? vp.width - 1 : xhi;
                yhi = yhi > vp.height - 1 ? vp.height - 1 : yhi;
                const int x0 = (int)(xlo / kTile), x1 = (int)(xhi / kTile) + 1;
                const int y0 = (int)(ylo / kTile), y1 = (int)(yhi / kTile) + 1;
                rc = make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)x1, (unsigned short)y1);
                tiles = (uint32_t)((x1 - x0) * (y1 - y0));
            }
        }

        Splat sp;
        sp.a = sp.b = sp.c = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tiles > 0) {
            const float uh = (float)g.u, vh = (float)g.v;
            sp.a = make_float4(uh, vh, (float)(g.u - (double)uh), (float)(g.v - (double)vh));
            sp.b = make_float4((float)g.A, (float)g.B, (float)g.C, opacity);
            // view direction from the camera centre
            float dx = mxf - vp.campos[0], dy = myf - vp.campos[1], dz = mzf - vp.campos[2];
            const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
            dx *= inv;
            dy *= inv;
            dz *= inv;
            float Y[16];
            sh_basis(dx, dy, dz, DEG, Y);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < ncoef; ++k) acc += coef[k * 3 + ch] * Y[k];
                col[ch] = fmaxf(acc + 0.5f, 0.0f);
            }
            sp.c = make_float4(col[0], col[1], col[2], (float)g.tz);
        }
        bool changed = false;
        if (valid) {
            const int64_t o = (int64_t)v * n + i;
            float4* dst = reinterpret_cast<float4*>(a.splats + o);
            dst[0] = sp.a;
            dst[1] = sp.b;
            dst[2] = sp.c;
            const uint32_t key = keyed ? __float_as_uint((float)tz_key) : 0xFFFFFFFFu;
            if (a.changed) {
                const uint32_t key0 = a.depth_key[o];
                const ushort4 rc0 = a.rect[o];
                changed = key0 != key || rc0.x != rc.x || rc0.y != rc.y || rc0.z != rc.z || rc0.w != rc.w;
            }
            a.depth_key[o] = key;
            a.radius[o] = tiles > 0 ? g.radius : 0;
            a.tiles_touched[o] = tiles;
            a.rect[o] = rc;
        }

        // per-block visible count and pair total of the view (no atomics: a
        // single counter hit by every wave serialises); reduce_partials_kernel
        // sums them
        const uint64_t vis = __ballot(tiles > 0);
        const uint64_t front = __ballot(valid && keyed);
        const uint64_t moved = __ballot(changed);
        uint32_t wave_pairs = tiles;
        for (int o = 32; o > 0; o >>= 1) wave_pairs += __shfl_xor(wave_pairs, o, 64);
        if ((threadIdx.x & 63) == 0) {
            s_vis[threadIdx.x >> 6] = (uint32_t)__popcll(vis);
            s_pairs[threadIdx.x >> 6] = wave_pairs;
            s_front[threadIdx.x >> 6] = (uint32_t)__popcll(front);
            s_changed[threadIdx.x >> 6] = (uint32_t)__popcll(moved);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t* pp = a.partials + 4 * (blk * a.n_views + v);
            pp[0] = s_vis[0] + s_vis[1] + s_vis[2] + s_vis[3];
            pp[1] = s_pairs[0] + s_pairs[1] + s_pairs[2] + s_pairs[3];
            pp[2] = s_front[0] + s_front[1] + s_front[2] + s_front[3];
            pp[3] = s_changed[0] + s_changed[1] + s_changed[2] + s_changed[3];
        }
        __syncthreads();   // s_vis / s_pairs are reused by the next view
    }
}

// ---------------------------------------------------------------- backward
// Gradient of the projection from the per-item gradient of the blend's inputs
// g9 = dL/d(u, v, A, B, C, opacity, r, g, b), summed over the views that show
// the Gaussian.  The forward quantities are recomputed (an item with tiles was
// visible in its view, so every cull passed).  Two kernels: the colour (SH)
// part in float and the geometry part in double precision, so that neither
// holds the other's registers.

// d(real SH basis Y_k)/d(x, y, z), k < (deg+1)^2, of the polynomial forms
// that sh_basis evaluates (equal to the basis on the unit sphere; only the
// tangential part of this gradient is used)
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int k, float& gx, float& gy, float& gz)
{
    const float c1 = 0.48860251190291992f, k4 = 1.0925484305920792f, k6 = 0.31539156525252005f,
                k8 = 0.54627421529603959f, k9 = 0.59004358992664352f, k10 = 2.8906114426405538f,
                k11 = 0.45704579946446572f, k12 = 0.37317633259011540f, k14 = 1.4453057213202769f;
    gx = gy = gz = 0.0f;
    switch (k) {
    case 1: gy = -c1; break;
    case 2: gz = c1; break;
    case 3: gx = -c1; break;
    case 4: gx = k4 * y; gy = k4 * x; break;
    case 5: gy = -k4 * z; gz = -k4 * y; break;
    case 6: gx = -2.0f * k6 * x; gy = -2.0f * k6 * y; gz = 4.0f * k6 * z; break;
    case 7: gx = -k4 * z; gz = -k4 * x; break;
    case 8: gx = 2.0f * k8 * x; gy = -2.0f * k8 * y; break;
    case 9: gx = -6.0f * k9 * x * y; gy = -3.0f * k9 * (x * x - y * y); break;
    case 10: gx = k10 * y * z; gy = k10 * x * z; gz = k10 * x * y; break;
    case 11: gx = 2.0f * k11 * x * y; gy = -k11 * (4.0f * z * z - x * x - 3.0f * y * y); gz = -8.0f * k11 * y * z; break;
    case 12: gx = -6.0f * k12 * x * z; gy = -6.0f * k12 * y * z; gz = k12 * (6.0f * z * z - 3.0f * x * x - 3.0f * y * y); break;
    case 13: gx = -k11 * (4.0f * z * z - 3.0f * x * x - y * y); gy = 2.0f * k11 * x * y; gz = -8.0f * k11 * x * z; break;
    case 14: gx = 2.0f * k14 * x * z; gy = -2.0f * k14 * y * z; gz = k14 * (x * x - y * y); break;
    case 15: gx = -3.0f * k9 * (x * x - y * y); gy = 6.0f * k9 * x * y; break;
    default: break;
    }
}

// Colour part of the backward, one thread per Gaussian, in float as the
// forward evaluates it: rgb_c = max(0, sum_k f_kc Y_k(d) + 0.5) with d the
// unit view direction.  Writes the SH coefficient gradients (summed over the
// views, zero where no view shows the Gaussian) and the mean's gradient
// through d; the geometry kernel adds the rest of the mean's gradient
// afterwards.  Channels outer, views inner: only one channel's coefficients
// and gradient sums are live, and d and Y(d) are recomputed per channel (a few
// dozen flops) rather than held.  The mean's gradient through d is linear in
// dL/dY = sum_c gc_c f_kc, so it is summed channel by channel.
template <int DT, int DEG>
__global__ __launch_bounds__(256) void project_backward_color_kernel(ProjectBackArgs a)
{
    constexpr int ncoef = (DEG + 1) * (DEG + 1);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    const float mx = a.means[i], my = a.means[n + i], mz = a.means[2 * n + i];
    float gm0 = 0.0f, gm1 = 0.0f, gm2 = 0.0f;
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        float f[ncoef], gf[ncoef];
#pragma unroll
        for (int k = 0; k < ncoef; ++k) {
            f[k] = load_attr<DT>(a.sh, (int64_t)(k * 3 + ch) * n + i);
            gf[k] = 0.0f;
        }
        for (int v = 0; v < a.n_views; ++v) {
            const int64_t item = (int64_t)v * n + i;
            if (a.tiles_touched[item] == 0) continue;
            const ViewParams& vp = a.views[v];
            float dx = mx - vp.campos[0], dy = my - vp.campos[1], dz = mz - vp.campos[2];
            const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
            dx *= inv;
            dy *= inv;
            dz *= inv;
            float Y[16];
            sh_basis(dx, dy, dz, DEG, Y);
            float raw = 0.0f;   // the forward's colour sum
#pragma unroll
            for (int k = 0; k < ncoef; ++k) raw += f[k] * Y[k];
            if (!(raw + 0.5f > 0.0f)) continue;   // clamped at 0: no gradient
            const float gc = a.grad2d[item * kGrad2d + 6 + ch];
            float gd0 = 0.0f, gd1 = 0.0f, gd2 = 0.0f;
#pragma unroll
            for (int k = 0; k < ncoef; ++k) {
                gf[k] += gc * Y[k];
                if (k > 0) {
                    float hx, hy, hz;
                    sh_basis_grad(dx, dy, dz, k, hx, hy, hz);
                    const float gy = gc * f[k];
                    gd0 += gy * hx;
                    gd1 += gy * hy;
                    gd2 += gy * hz;
                }
            }
            // d = (m - campos) / |m - campos|: the tangential part over the length
            const float dot = dx * gd0 + dy * gd1 + dz * gd2;
            gm0 += (gd0 - dx * dot) * inv;
            gm1 += (gd1 - dy * dot) * inv;
            gm2 += (gd2 - dz * dot) * inv;
        }
#pragma unroll
        for (int k = 0; k < ncoef; ++k) a.g_sh[(int64_t)(k * 3 + ch) * n + i] = gf[k];
    }
    a.g_means[i] = gm0;
    a.g_means[n + i] = gm1;
    a.g_means[2 * n + i] = gm2;
}

// Geometry part, one thread per Gaussian, in double precision: from
// dL/d(u, v, A, B, C, opacity) of every view through the conic inverse, the
// EWA Jacobian (guard-band clamp included), the world covariance, the scales,
// the normalised quaternion and the sigmoid.  Adds to the mean's gradient
// that the colour kernel wrote.
template <int DT, bool kOneView>
__global__ __launch_bounds__(256) void project_backward_geometry_kernel(ProjectBackArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    const double mx = a.means[i], my = a.means[n + i], mz = a.means[2 * n + i];
    const double l[3] = {load_attr<DT>(a.log_scales, i), load_attr<DT>(a.log_scales, n + i),
                         load_attr<DT>(a.log_scales, 2 * n + i)};
    const double q4[4] = {load_attr<DT>(a.quats, i), load_attr<DT>(a.quats, n + i), load_attr<DT>(a.quats, 2 * n + i),
                          load_attr<DT>(a.quats, 3 * n + i)};
    const float logit = load_attr<DT>(a.logits, i);

    // rotation Q of the unit quaternion, scales, M = Q diag(s), Sg = M M^T
    const double qn = sqrt(((q4[0] * q4[0] + q4[1] * q4[1]) + q4[2] * q4[2]) + q4[3] * q4[3]);
    double gm[3] = {0, 0, 0}, gQ[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gsc[3] = {0, 0, 0}, gop = 0.0;
    double Sg[9];
    const bool cov_ok = world_covariance(l[0], l[1], l[2], q4[0], q4[1], q4[2], q4[3], Sg);
    const double inv_qn = cov_ok ? 1.0 / qn : 0.0;
    const double w = q4[0] * inv_qn, x = q4[1] * inv_qn, y = q4[2] * inv_qn, z = q4[3] * inv_qn;
    double Q[9];
    Q[0] = 1.0 - 2.0 * (y * y + z * z);
    Q[1] = 2.0 * (x * y - w * z);
    Q[2] = 2.0 * (x * z + w * y);
    Q[3] = 2.0 * (x * y + w * z);
    Q[4] = 1.0 - 2.0 * (x * x + z * z);
    Q[5] = 2.0 * (y * z - w * x);
    Q[6] = 2.0 * (x * z - w * y);
    Q[7] = 2.0 * (y * z + w * x);
    Q[8] = 1.0 - 2.0 * (x * x + y * y);
    const double sc[3] = {exp(l[0]), exp(l[1]), exp(l[2])};

    const int n_views = kOneView ? 1 : a.n_views;
    for (int v = 0; cov_ok && v < n_views; ++v) {
        const int64_t item = (int64_t)v * n + i;
        if (a.tiles_touched[item] == 0) continue;
        const float* g9 = a.grad2d + item * kGrad2d;
        const ViewParams& vp = a.views[v];
        const double gu = g9[0], gv = g9[1], gA = g9[2], gB = g9[3], gC = g9[4];
        gop += g9[5];
        const double* W = vp.R;
        const double t0 = ((W[0] * mx + W[1] * my) + W[2] * mz) + vp.t[0];
        const double t1 = ((W[3] * mx + W[4] * my) + W[5] * mz) + vp.t[1];
        const double t2 = ((W[6] * mx + W[7] * my) + W[8] * mz) + vp.t[2];
        // V = W Sg W^T
        double L[9], V[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) L[3 * r + c] = W[3 * r] * Sg[c] + W[3 * r + 1] * Sg[3 + c] + W[3 * r + 2] * Sg[6 + c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) V[3 * r + c] = L[3 * r] * W[3 * c] + L[3 * r + 1] * W[3 * c + 1] + L[3 * r + 2] * W[3 * c + 2];
        const double fx = vp.fx, fy = vp.fy;
        const double limx = 1.3 * ((0.5 * (double)vp.width) / fx), limy = 1.3 * ((0.5 * (double)vp.height) / fy);
        const double rx = t0 / t2, ry = t1 / t2;   // divided as the forward divides: same clamp decisions
        const bool clx = rx < -limx || rx > limx, cly = ry < -limy || ry > limy;
        const double xcl = fmin(limx, fmax(-limx, rx)) * t2, ycl = fmin(limy, fmax(-limy, ry)) * t2;
        const double it = 1.0 / t2, it2 = it * it, it3 = it2 * it;
        const double J[6] = {fx * it, 0.0, -(fx * xcl) * it2, 0.0, fy * it, -(fy * ycl) * it2};
        double JV[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) JV[3 * r + c] = J[3 * r] * V[c] + J[3 * r + 1] * V[3 + c] + J[3 * r + 2] * V[6 + c];
        const double ca = (JV[0] * J[0] + JV[1] * J[1] + JV[2] * J[2]) + 0.3;
        const double cb = JV[0] * J[3] + JV[1] * J[4] + JV[2] * J[5];
        const double cc = (JV[3] * J[3] + JV[4] * J[4] + JV[5] * J[5]) + 0.3;
        const double idet = 1.0 / (ca * cc - cb * cb);
        const double A = cc * idet, B = -cb * idet, C = ca * idet;
        // conic -> 2D covariance: dL/dSigma'' = -Q G Q with G = [[gA, gB/2], [gB/2, gC]]
        const double G01 = 0.5 * gB;
        const double QG00 = A * gA + B * G01, QG01 = A * G01 + B * gC, QG10 = B * gA + C * G01, QG11 = B * G01 + C * gC;
        const double gP00 = -(QG00 * A + QG01 * B), gP01 = -(QG00 * B + QG01 * C), gP11 = -(QG10 * B + QG11 * C);
        // Sigma' = J V J^T: gV = J^T gP J, gJ = 2 gP J V (gP, V symmetric)
        const double gP[4] = {gP00, gP01, gP01, gP11};
        double gV[9], gJ[6];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                gV[3 * r + c] = J[r] * (gP[0] * J[c] + gP[1] * J[3 + c]) + J[3 + r] * (gP[2] * J[c] + gP[3] * J[3 + c]);
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) gJ[3 * r + c] = 2.0 * (gP[2 * r] * JV[c] + gP[2 * r + 1] * JV[3 + c]);
        // camera-space position t: through J, and through the centre (u, v)
        double gt0 = gu * fx * it, gt1 = gv * fy * it;
        double gt2 = -(gu * fx * t0 + gv * fy * t1) * it2;
        gt2 += -(gJ[0] * fx + gJ[4] * fy) * it2;
        if (!clx) {
            gt0 += -gJ[2] * fx * it2;
            gt2 += gJ[2] * 2.0 * fx * t0 * it3;
        } else {
            gt2 += gJ[2] * fx * xcl * it3;
        }
        if (!cly) {
            gt1 += -gJ[5] * fy * it2;
            gt2 += gJ[5] * 2.0 * fy * t1 * it3;
        } else {
            gt2 += gJ[5] * fy * ycl * it3;
        }
        for (int c = 0; c < 3; ++c) gm[c] += W[c] * gt0 + W[3 + c] * gt1 + W[6 + c] * gt2;
        // V = W Sg W^T -> gSg = W^T gV W; Sg = M M^T -> gM = 2 gSg M; M = Q diag(s)
        double gW1[9], gSg[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) gW1[3 * r + c] = gV[3 * r] * W[c] + gV[3 * r + 1] * W[3 + c] + gV[3 * r + 2] * W[6 + c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) gSg[3 * r + c] = W[r] * gW1[c] + W[3 + r] * gW1[3 + c] + W[6 + r] * gW1[6 + c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double gM = 0.0;
                for (int k = 0; k < 3; ++k) gM += 2.0 * gSg[3 * r + k] * Q[3 * k + c] * sc[c];
                gQ[3 * r + c] += gM * sc[c];
                gsc[c] += gM * Q[3 * r + c];
            }
    }

    // quaternion: through the rotation matrix of q / |q|
    double gw = 2.0 * (-z * gQ[1] + y * gQ[2] + z * gQ[3] - x * gQ[5] - y * gQ[6] + x * gQ[7]);
    double gx = 2.0 * (y * gQ[1] + z * gQ[2] + y * gQ[3] - 2.0 * x * gQ[4] - w * gQ[5] + z * gQ[6] + w * gQ[7] -
                       2.0 * x * gQ[8]);
    double gy = 2.0 * (-2.0 * y * gQ[0] + x * gQ[1] + w * gQ[2] + x * gQ[3] + z * gQ[5] - w * gQ[6] + z * gQ[7] -
                       2.0 * y * gQ[8]);
    double gz = 2.0 * (-2.0 * z * gQ[0] - w * gQ[1] + x * gQ[2] + w * gQ[3] - 2.0 * z * gQ[4] + y * gQ[5] + x * gQ[6] +
                       y * gQ[7]);
    const double qd = w * gw + x * gx + y * gy + z * gz;
    a.g_quats[i] = (float)((gw - w * qd) * inv_qn);
    a.g_quats[n + i] = (float)((gx - x * qd) * inv_qn);
    a.g_quats[2 * n + i] = (float)((gy - y * qd) * inv_qn);
    a.g_quats[3 * n + i] = (float)((gz - z * qd) * inv_qn);
    for (int c = 0; c < 3; ++c) {
        a.g_means[(int64_t)c * n + i] = (float)((double)a.g_means[(int64_t)c * n + i] + gm[c]);
        a.g_log_scales[(int64_t)c * n + i] = (float)(gsc[c] * sc[c]);
    }
    const double sig = 1.0 / (1.0 + exp(-(double)logit));
    a.g_logits[i] = (float)(gop * sig * (1.0 - sig));
}

template <int DT>
void launch_project_backward_dt(const ProjectBackArgs& a, unsigned blocks, hipStream_t s)
{
    switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL((project_backward_color_kernel<DT, 0>), dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((project_backward_color_kernel<DT, 1>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((project_backward_color_kernel<DT, 2>), dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((project_backward_color_kernel<DT, 3>), dim3(blocks), dim3(256), 0, s, a); break;
    }
    // one view: no loop, fewer live registers in the geometry kernel
    if (a.n_views == 1) hipLaunchKernelGGL((project_backward_geometry_kernel<DT, true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((project_backward_geometry_kernel<DT, false>), dim3(blocks), dim3(256), 0, s, a);
}

}  // namespace

// Per view (one block each): Gaussians on screen, pairs and Gaussians with a
// depth key (past the culls), summed over the projection blocks' partials.
// With changed, also the items whose key or rectangle changed (added over
// the views; each view's share clamped to 2^32 - 1), clearing the flag that
// none did when any did.
__global__ __launch_bounds__(1024) void reduce_partials_kernel(const uint32_t* __restrict__ partials, int blocks,
                                                               int n_views, uint32_t* view_counts, uint32_t* changed)
{
    // 64-bit sums: in each thread over a stride of blocks, in each wave by
    // shuffles, then over the 16 waves in LDS
    __shared__ unsigned long long sv[16], sp[16], sf[16], sc[16];
    const int v = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long vis = 0, pairs = 0, front = 0, moved = 0;
#pragma unroll 4
    for (int b = threadIdx.x; b < blocks; b += 1024) {
        const uint4 pp = *reinterpret_cast<const uint4*>(partials + 4 * ((int64_t)b * n_views + v));
        vis += pp.x;
        pairs += pp.y;
        front += pp.z;
        moved += changed ? pp.w : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) {
        vis += __shfl_xor(vis, o, 64);
        pairs += __shfl_xor(pairs, o, 64);
        front += __shfl_xor(front, o, 64);
        moved += __shfl_xor(moved, o, 64);
    }
    if (lane == 0) {
        sv[wave] = vis;
        sp[wave] = pairs;
        sf[wave] = front;
        sc[wave] = moved;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tv = 0, tp = 0, tf = 0, tc = 0;
        for (int w = 0; w < 16; ++w) {
            tv += sv[w];
            tp += sp[w];
            tf += sf[w];
            tc += sc[w];
        }
        uint32_t* c = view_counts + (int64_t)kViewCounters * v;
        c[0] = (uint32_t)tv;
        c[1] = (uint32_t)tf;
        c[2] = (uint32_t)tp;
        c[3] = (uint32_t)(tp >> 32);
        if (changed && tc > 0) {
            // views add their counts; any change clears the flag (all
            // writers store the same 0)
            atomicAdd(&changed[0], tc > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tc);
            changed[1] = 0u;
        }
    }
}

template <int DT, bool kOneView>
void launch_project_dt(const ProjectArgs& a, unsigned blocks, hipStream_t s)
{
    switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL((project_kernel<DT, 0, kOneView>), dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((project_kernel<DT, 1, kOneView>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((project_kernel<DT, 2, kOneView>), dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((project_kernel<DT, 3, kOneView>), dim3(blocks), dim3(256), 0, s, a); break;
    }
}

template <int DT>
void launch_project_views(const ProjectArgs& a, unsigned blocks, hipStream_t s)
{
    if (a.n_views == 1) launch_project_dt<DT, true>(a, blocks, s);
    else launch_project_dt<DT, false>(a, blocks, s);
}

hipError_t launch_project_backward(const ProjectBackArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.n + 255) / 256);
    switch (a.dtype) {
    case 0: launch_project_backward_dt<0>(a, blocks, s); break;
    case 1: launch_project_backward_dt<1>(a, blocks, s); break;
    default: launch_project_backward_dt<2>(a, blocks, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_project(const ProjectArgs& a, hipStream_t s)
{
    if (a.n_views <= 0) return hipSuccess;
    if (a.n == 0) return launch_fill_u32(a.view_counts, 0u, (int64_t)kViewCounters * a.n_views, s);
    const unsigned blocks = (unsigned)((a.n + 255) / 256);
    const unsigned grid = blocks + (a.order ? 1u : 0u);   // the order's workgroup first
    switch (a.dtype) {
    case 0: launch_project_views<0>(a, grid, s); break;
    case 1: launch_project_views<1>(a, grid, s); break;
    default: launch_project_views<2>(a, grid, s); break;
    }
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)a.n_views), dim3(1024), 0, s,
                       (const uint32_t*)a.partials, (int)blocks, a.n_views, a.view_counts,
                       a.changed);
    return hipGetLastError();
}

}  // namespace gsmi
