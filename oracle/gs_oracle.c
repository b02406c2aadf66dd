/*
 * gs_oracle.c -- plain FP64 CPU oracle for the 3D Gaussian Splatting forward
 * render (cull, project, sort, composite; Sec. 3.1 and Eq. 1 of "Rendering 3D
 * Gaussians on a Graph Processor").
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke entry point and the CPU
 * baseline leg of bench.py may load this library.  It shares no code, header
 * or constant table with the HIP library: everything below is written from
 * the paper's definitions and the readings listed at each function.
 *
 * Built with: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA
 * contraction, so every expression rounds exactly as written).
 *
 * Conventions (readings of points the paper leaves open):
 *   - arrays are structure-of-arrays, channel-major: x[c*n + i];
 *   - camera R (row-major) and t map world to camera space, x right, y down,
 *     z forward; pixel (px, py) samples the image point (px, py);
 *   - the projection geometry (camera-space position, covariance, conic,
 *     bounding radius, 2D mean) is defined in IEEE double precision with the
 *     operation order written below; the sort key uses the float32 rounding of
 *     the camera-space depth;
 *   - every input array holds float32 values, promoted exactly to double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16

typedef struct {
    double R[9], t[3];
    double fx, fy, cx, cy, near_plane;
    int width, height;
} camera_t;

/* cam17 = R[9], t[3], fx, fy, cx, cy, near (float32). */
static camera_t load_camera(const float* cam17, int width, int height)
{
    camera_t c;
    for (int k = 0; k < 9; ++k) c.R[k] = cam17[k];
    for (int k = 0; k < 3; ++k) c.t[k] = cam17[9 + k];
    c.fx = cam17[12]; c.fy = cam17[13]; c.cx = cam17[14]; c.cy = cam17[15];
    c.near_plane = cam17[16];
    c.width = width; c.height = height;
    return c;
}

/* ---------------------------------------------------------------------------
 * Real spherical-harmonic basis up to degree 3, in the index order
 * k = l*l + l + m (m = -l..l).  Definition: with the complex orthonormal
 * harmonics Y_l^m(theta, phi) that carry the Condon-Shortley phase,
 *   Y_{l,m} = sqrt(2) Im Y_l^{|m|}  (m < 0),  Y_l^0  (m = 0),
 *   Y_{l,m} = sqrt(2) Re Y_l^m      (m > 0),
 * where x = sin(theta)cos(phi), y = sin(theta)sin(phi), z = cos(theta) is the
 * unit direction.  Written out from the associated Legendre functions
 * P_l^m(z) (which include the (-1)^m phase).  Sec. 3.1: view-dependent colour
 * is encoded with spherical harmonics.
 * ------------------------------------------------------------------------- */
void or_sh_basis(const double d[3], double out[16])
{
    const double pi = 3.14159265358979323846;
    double x = d[0], y = d[1], z = d[2];
    out[0] = 0.5 * sqrt(1.0 / pi);
    /* l = 1: P_1^1 = -sin(theta) */
    double c1 = sqrt(3.0 / (4.0 * pi));
    out[1] = -c1 * y;
    out[2] = c1 * z;
    out[3] = -c1 * x;
    /* l = 2: P_2^1 = -3 z sin, P_2^2 = 3 sin^2 */
    out[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    out[5] = -0.5 * sqrt(15.0 / pi) * y * z;
    out[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    out[7] = -0.5 * sqrt(15.0 / pi) * x * z;
    out[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    /* l = 3: P_3^1 = -(3/2)(5z^2-1) sin, P_3^2 = 15 z sin^2, P_3^3 = -15 sin^3 */
    out[9]  = -0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    out[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    out[11] = -0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    out[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    out[13] = -0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    out[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    out[15] = -0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

/* ---------------------------------------------------------------------------
 * Per-Gaussian geometry (Sec. 3.1 stages 1-2, the 3-sigma bound of Sec. 4.4).
 * Fills the intermediates for one Gaussian; returns 0 when it is culled.
 * ------------------------------------------------------------------------- */
typedef struct {
    double tcam[3];      /* camera-space centre */
    double Rq[9];        /* rotation of the normalised quaternion */
    double Sigma[9];     /* world covariance R S S^T R^T */
    double V[9];         /* camera-space covariance W Sigma W^T */
    double J[6];         /* 2x3 Jacobian of the perspective map */
    double cov2d[3];     /* J V J^T + 0.3 I  as (a, b, c) */
    double conic[3];     /* inverse of cov2d as (A, B, C) */
    double lambda_max;
    double radius3;      /* 3 sqrt(lambda_max) before rounding up */
    int32_t radius;
    double u, v;         /* projected centre in pixels */
} geom_t;

static int geometry(const camera_t* c, const double mu[3], const double ls[3],
                    const double q[4], geom_t* g)
{
    const double* W = c->R;
    /* stage 1: camera space and the near-plane cull (Sec. 4.5 culling) */
    for (int r = 0; r < 3; ++r)
        g->tcam[r] = ((W[3 * r] * mu[0] + W[3 * r + 1] * mu[1]) + W[3 * r + 2] * mu[2]) + c->t[r];
    double tx = g->tcam[0], ty = g->tcam[1], tz = g->tcam[2];
    if (!(tz > c->near_plane) || !isfinite(tx) || !isfinite(ty) || !isfinite(tz)) return 0;

    /* rotation from the quaternion (w, x, y, z), normalised first */
    double n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    if (!(n2 > 0.0) || !isfinite(n2)) return 0;
    double s = sqrt(n2);
    double w = q[0] / s, x = q[1] / s, y = q[2] / s, z = q[3] / s;
    double* Rq = g->Rq;
    Rq[0] = 1.0 - 2.0 * (y * y + z * z); Rq[1] = 2.0 * (x * y - w * z);       Rq[2] = 2.0 * (x * z + w * y);
    Rq[3] = 2.0 * (x * y + w * z);       Rq[4] = 1.0 - 2.0 * (x * x + z * z); Rq[5] = 2.0 * (y * z - w * x);
    Rq[6] = 2.0 * (x * z - w * y);       Rq[7] = 2.0 * (y * z + w * x);       Rq[8] = 1.0 - 2.0 * (x * x + y * y);

    /* Sigma = (R S)(R S)^T with S = diag(exp(log_scale)) (Sec. 3.1) */
    double S[3] = {exp(ls[0]), exp(ls[1]), exp(ls[2])};
    double M[9];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) M[3 * j + k] = Rq[3 * j + k] * S[k];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            g->Sigma[3 * j + k] = (M[3 * j] * M[3 * k] + M[3 * j + 1] * M[3 * k + 1]) + M[3 * j + 2] * M[3 * k + 2];

    /* V = W Sigma W^T, left product first */
    double A[9];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            A[3 * j + k] = (W[3 * j] * g->Sigma[k] + W[3 * j + 1] * g->Sigma[3 + k]) + W[3 * j + 2] * g->Sigma[6 + k];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            g->V[3 * j + k] = (A[3 * j] * W[3 * k] + A[3 * j + 1] * W[3 * k + 1]) + A[3 * j + 2] * W[3 * k + 2];

    /* Jacobian of (fx x/z + cx, fy y/z + cy), evaluated with x/z and y/z
     * clamped to 1.3 times the half-image tangent (guard band) */
    double limx = 1.3 * ((0.5 * (double)c->width) / c->fx);
    double limy = 1.3 * ((0.5 * (double)c->height) / c->fy);
    double txtz = tx / tz, tytz = ty / tz;
    double xc = fmin(limx, fmax(-limx, txtz)) * tz;
    double yc = fmin(limy, fmax(-limy, tytz)) * tz;
    double* J = g->J;
    J[0] = c->fx / tz; J[1] = 0.0; J[2] = -(c->fx * xc) / (tz * tz);
    J[3] = 0.0; J[4] = c->fy / tz; J[5] = -(c->fy * yc) / (tz * tz);

    /* 2D covariance J V J^T plus the 0.3 px^2 low-pass of the EWA filter */
    double B[6];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 3; ++k)
            B[3 * j + k] = (J[3 * j] * g->V[k] + J[3 * j + 1] * g->V[3 + k]) + J[3 * j + 2] * g->V[6 + k];
    double P[4];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k)
            P[2 * j + k] = (B[3 * j] * J[3 * k] + B[3 * j + 1] * J[3 * k + 1]) + B[3 * j + 2] * J[3 * k + 2];
    double a = P[0] + 0.3, b = P[1], cc = P[3] + 0.3;
    g->cov2d[0] = a; g->cov2d[1] = b; g->cov2d[2] = cc;

    /* conic Q = inverse of the 2D covariance (Sec. 3.1, stage 2) */
    double det = a * cc - b * b;
    if (!(det > 0.0) || !isfinite(det)) return 0;
    g->conic[0] = cc / det; g->conic[1] = -b / det; g->conic[2] = a / det;

    /* bounding radius: three standard deviations of the larger eigenvalue
     * (Sec. 4.4), rounded up to whole pixels */
    double mid = 0.5 * (a + cc);
    double disc = mid * mid - det;
    g->lambda_max = mid + sqrt(fmax(0.0, disc));
    g->radius3 = 3.0 * sqrt(g->lambda_max);
    double r = ceil(g->radius3);
    if (!(r > 0.0) || !(r < 1e9)) return 0;
    g->radius = (int32_t)r;

    /* projected centre (unclamped x/z, y/z) */
    g->u = (c->fx * tx) / tz + c->cx;
    g->v = (c->fy * ty) / tz + c->cy;
    if (!isfinite(g->u) || !isfinite(g->v)) return 0;
    return 1;
}

/* Tiles overlapped by the square of half-width r pixels around (u, v): the
 * pixels x with |x - u| <= r and |y - v| <= r (Sec. 4.4's square bound).
 * Writes the tile rectangle [tx0, tx1) x [ty0, ty1); returns the tile count. */
static uint32_t tile_rect(double u, double v, int32_t r, int width, int height, int32_t rect[4])
{
    const double big = 1073741824.0; /* 2^30 keeps the integer span in range */
    double uc = fmin(big, fmax(-big, u)), vc = fmin(big, fmax(-big, v));
    int64_t xlo = (int64_t)ceil(uc) - r, xhi = (int64_t)floor(uc) + r;
    int64_t ylo = (int64_t)ceil(vc) - r, yhi = (int64_t)floor(vc) + r;
    rect[0] = rect[1] = rect[2] = rect[3] = 0;
    if (xhi < 0 || xlo > width - 1 || yhi < 0 || ylo > height - 1) return 0;
    if (xlo < 0) xlo = 0;
    if (ylo < 0) ylo = 0;
    if (xhi > width - 1) xhi = width - 1;
    if (yhi > height - 1) yhi = height - 1;
    rect[0] = (int32_t)(xlo / TILE); rect[2] = (int32_t)(xhi / TILE) + 1;
    rect[1] = (int32_t)(ylo / TILE); rect[3] = (int32_t)(yhi / TILE) + 1;
    return (uint32_t)((rect[2] - rect[0]) * (rect[3] - rect[1]));
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Debug view of one Gaussian's intermediates, for the pinning tests.
 * out: tcam[3] Rq[9] Sigma[9] V[9] J[6] cov2d[3] conic[3] lambda_max radius3
 *      radius u v   (= 47 doubles).  Returns 1 if not culled. */
int or_debug_geometry(const float* cam17, int width, int height, const double mu[3],
                      const double ls[3], const double q[4], double* out)
{
    camera_t c = load_camera(cam17, width, height);
    geom_t g;
    memset(&g, 0, sizeof g);
    int ok = geometry(&c, mu, ls, q, &g);
    double* o = out;
    memcpy(o, g.tcam, 3 * sizeof(double)); o += 3;
    memcpy(o, g.Rq, 9 * sizeof(double)); o += 9;
    memcpy(o, g.Sigma, 9 * sizeof(double)); o += 9;
    memcpy(o, g.V, 9 * sizeof(double)); o += 9;
    memcpy(o, g.J, 6 * sizeof(double)); o += 6;
    memcpy(o, g.cov2d, 3 * sizeof(double)); o += 3;
    memcpy(o, g.conic, 3 * sizeof(double)); o += 3;
    *o++ = g.lambda_max; *o++ = g.radius3; *o++ = g.radius; *o++ = g.u; *o++ = g.v;
    return ok;
}

/* ---------------------------------------------------------------------------
 * Projection of all Gaussians (Sec. 3.1 stages 1-2; colour of Sec. 3.1 with
 * the degree given; opacity sigma(alpha) of Eq. 1).
 *
 * Outputs (structure of arrays, n columns):
 *   mean2d[2][n], conic[3][n], opacity[n], rgb[3][n], depth[n]  (double)
 *   depth_bits[n]   bits of the float32 rounding of depth (the sort key)
 *   radius[n], rect[4][n] (tx0, ty0, tx1, ty1), tiles_touched[n]
 *   radius_margin[n] distance of 3 sqrt(lambda_max) to the nearest integer
 * A Gaussian that is culled or overlaps no tile has radius = 0,
 * tiles_touched = 0 and an all-zero rect.  Returns the number of Gaussians
 * that overlap at least one tile.
 * ------------------------------------------------------------------------- */
int64_t or_project(int64_t n, int sh_degree, const float* means, const float* log_scales,
                   const float* quats, const float* logits, const float* sh,
                   const float* cam17, int width, int height,
                   double* mean2d, double* conic, double* opacity, double* rgb, double* depth,
                   uint32_t* depth_bits, int32_t* radius, int32_t* rect, uint32_t* tiles_touched,
                   double* radius_margin)
{
    camera_t c = load_camera(cam17, width, height);
    int ncoef = (sh_degree + 1) * (sh_degree + 1);
    /* camera centre in world space: -R^T t */
    double campos[3];
    for (int k = 0; k < 3; ++k)
        campos[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
    int64_t visible = 0;
#pragma omp parallel for schedule(static) reduction(+ : visible)
    for (int64_t i = 0; i < n; ++i) {
        double mu[3] = {means[i], means[n + i], means[2 * n + i]};
        double ls[3] = {log_scales[i], log_scales[n + i], log_scales[2 * n + i]};
        double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
        geom_t g;
        int ok = geometry(&c, mu, ls, q, &g);
        int32_t rc[4] = {0, 0, 0, 0};
        uint32_t tiles = ok ? tile_rect(g.u, g.v, g.radius, width, height, rc) : 0;
        for (int k = 0; k < 4; ++k) rect[k * n + i] = rc[k];
        tiles_touched[i] = tiles;
        radius[i] = tiles ? g.radius : 0;
        radius_margin[i] = ok ? fabs(g.radius3 - nearbyint(g.radius3)) : INFINITY;
        if (!ok) {
            mean2d[i] = mean2d[n + i] = 0.0;
            conic[i] = conic[n + i] = conic[2 * n + i] = 0.0;
            opacity[i] = 0.0; rgb[i] = rgb[n + i] = rgb[2 * n + i] = 0.0;
            depth[i] = 0.0; depth_bits[i] = 0;
            continue;
        }
        visible += tiles ? 1 : 0;
        mean2d[i] = g.u; mean2d[n + i] = g.v;
        conic[i] = g.conic[0]; conic[n + i] = g.conic[1]; conic[2 * n + i] = g.conic[2];
        depth[i] = g.tcam[2];
        float df = (float)g.tcam[2];
        memcpy(&depth_bits[i], &df, 4);
        opacity[i] = sigmoid((double)logits[i]);
        /* colour: SH evaluated along the unit direction from the camera centre */
        double d[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        d[0] /= len; d[1] /= len; d[2] /= len;
        double Y[16];
        or_sh_basis(d, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < ncoef; ++k) acc += (double)sh[((int64_t)k * 3 + ch) * n + i] * Y[k];
            acc += 0.5;
            rgb[ch * n + i] = acc > 0.0 ? acc : 0.0;
        }
    }
    return visible;
}

/* ---------------------------------------------------------------------------
 * Binning and sort.  Each overlapped tile of Gaussian i gives one pair
 * key = (tile_id << 32) | depth_bits[i], value = i, emitted in the order of
 * i, then tile row, then tile column; tile_id = ty * tiles_x + tx.
 * ------------------------------------------------------------------------- */
typedef struct { uint64_t key; uint32_t value; uint32_t pad; } pair_t;

static int cmp_pair(const void* a, const void* b)
{
    const pair_t* p = (const pair_t*)a;
    const pair_t* q = (const pair_t*)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->value != q->value) return p->value < q->value ? -1 : 1;
    return 0;
}

/* Emits the K pairs in emission order.  offsets[n] receives the exclusive
 * prefix sum of tiles_touched.  Returns K. */
int64_t or_emit_pairs(int64_t n, const int32_t* rect, const uint32_t* tiles_touched,
                      const uint32_t* depth_bits, int tiles_x, uint64_t* offsets,
                      uint64_t* keys, uint32_t* values)
{
    uint64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        offsets[i] = k;
        if (tiles_touched[i] == 0) continue;
        for (int32_t ty = rect[n + i]; ty < rect[3 * n + i]; ++ty)
            for (int32_t tx = rect[i]; tx < rect[2 * n + i]; ++tx) {
                uint64_t tile = (uint64_t)ty * (uint64_t)tiles_x + (uint64_t)tx;
                keys[k] = (tile << 32) | depth_bits[i];
                values[k] = (uint32_t)i;
                ++k;
            }
    }
    return (int64_t)k;
}

/* Sorts the pairs by (key, value), ascending (the library qsort is the sort). */
void or_sort_pairs(int64_t K, uint64_t* keys, uint32_t* values)
{
    pair_t* p = (pair_t*)malloc((size_t)(K > 0 ? K : 1) * sizeof(pair_t));
    for (int64_t j = 0; j < K; ++j) { p[j].key = keys[j]; p[j].value = values[j]; p[j].pad = 0; }
    qsort(p, (size_t)K, sizeof(pair_t), cmp_pair);
    for (int64_t j = 0; j < K; ++j) { keys[j] = p[j].key; values[j] = p[j].value; }
    free(p);
}

/* ranges[t] = [start, end) of tile t in the sorted key list. */
void or_tile_ranges(int64_t K, const uint64_t* keys, int64_t num_tiles, uint64_t* ranges)
{
    for (int64_t t = 0; t < num_tiles; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
    for (int64_t j = 0; j < K; ++j) {
        uint64_t t = keys[j] >> 32;
        if (j == 0 || (keys[j - 1] >> 32) != t) ranges[2 * t] = (uint64_t)j;
        ranges[2 * t + 1] = (uint64_t)j + 1;
    }
}

/* Per-tile counts of pairs, straight from the rectangles. */
void or_tile_counts(int64_t n, const int32_t* rect, const uint32_t* tiles_touched,
                    int tiles_x, int64_t num_tiles, uint64_t* counts)
{
    for (int64_t t = 0; t < num_tiles; ++t) counts[t] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (tiles_touched[i] == 0) continue;
        for (int32_t ty = rect[n + i]; ty < rect[3 * n + i]; ++ty)
            for (int32_t tx = rect[i]; tx < rect[2 * n + i]; ++tx)
                counts[(int64_t)ty * tiles_x + tx] += 1;
    }
}

typedef struct { uint32_t bits; uint32_t index; } depth_entry_t;

static int cmp_depth_entry(const void* a, const void* b)
{
    const depth_entry_t* p = (const depth_entry_t*)a;
    const depth_entry_t* q = (const depth_entry_t*)b;
    if (p->bits != q->bits) return p->bits < q->bits ? -1 : 1;
    if (p->index != q->index) return p->index < q->index ? -1 : 1;
    return 0;
}

/* The sorted list of one tile: every Gaussian whose rectangle holds the tile,
 * ordered by (depth_bits, index).  Writes at most cap values; returns the
 * list length. */
int64_t or_tile_list(int64_t n, const int32_t* rect, const uint32_t* tiles_touched,
                     const uint32_t* depth_bits, int tiles_x, int64_t tile,
                     uint32_t* out, int64_t cap)
{
    int32_t tx = (int32_t)(tile % tiles_x), ty = (int32_t)(tile / tiles_x);
    int64_t m = 0, alloc = 1024;
    depth_entry_t* e = (depth_entry_t*)malloc((size_t)alloc * sizeof(depth_entry_t));
    for (int64_t i = 0; i < n; ++i) {
        if (tiles_touched[i] == 0) continue;
        if (tx < rect[i] || tx >= rect[2 * n + i] || ty < rect[n + i] || ty >= rect[3 * n + i]) continue;
        if (m == alloc) { alloc *= 2; e = (depth_entry_t*)realloc(e, (size_t)alloc * sizeof(depth_entry_t)); }
        e[m].bits = depth_bits[i];
        e[m].index = (uint32_t)i;
        ++m;
    }
    qsort(e, (size_t)m, sizeof(depth_entry_t), cmp_depth_entry);
    for (int64_t j = 0; j < m && j < cap; ++j) out[j] = e[j].index;
    free(e);
    return m;
}

/* ---------------------------------------------------------------------------
 * Front-to-back compositing of one pixel along a depth-ordered list (Eq. 1
 * with the EWA falloff, per-pixel walk of Sec. 4.5), with the thresholds read
 * as: alpha = min(0.99, sigma * exp(power)); entries with alpha < 1/255 are
 * skipped; the walk stops before an entry that would take the transmittance
 * below 1e-4.
 *   out5 = (r, g, b, final T, n_contrib) where n_contrib is one past the list
 *   position of the last entry that contributed (0 if none).
 *   margins2 = how far the two kinds of threshold decision met on the walk
 *   sit from their thresholds, in units of a float32 error bound (a value
 *   below 1 means a float32 evaluation may take the other branch):
 *     alpha:  |255 a - 1| / e_a with e_a = 16u (1 + S), u = 2^-24 and
 *             S = (|A| dx^2 + |C| dy^2)/2 + |B dx dy|, the size of the terms
 *             of the quadratic form (it bounds the cancellation error); a
 *             float32 evaluation with relative error 2u in dx, dy, 3u in the
 *             conic and opacity and 2u in exp2 stays within half of e_a;
 *             an alpha clamped to 0.99 carries only the 2u of that constant;
 *     T:      |T' / 1e-4 - 1| / e_T with e_T the accumulated relative error
 *             bound of T': each factor 1 - a contributes (e_a / 2) a / (1 - a)
 *             (the alpha bound above) plus u (one rounding of T (1 - a)).
 * ------------------------------------------------------------------------- */
static void composite_pixel(double px, double py, const uint32_t* list, int64_t len, int64_t n,
                            const double* mean2d, const double* conic, const double* opacity,
                            const double* rgb, const double bg[3], double out5[5], double margins2[2])
{
    const double u = 1.0 / 16777216.0;
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    double eT = 0.0;
    double m_alpha = INFINITY, m_T = INFINITY;
    int64_t last = 0;
    for (int64_t j = 0; j < len; ++j) {
        int64_t i = list[j];
        double dx = mean2d[i] - px, dy = mean2d[n + i] - py;
        double qa = conic[i] * dx * dx, qc = conic[2 * n + i] * dy * dy, qb = conic[n + i] * dx * dy;
        double power = -0.5 * (qa + qc) - qb;
        double a = opacity[i] * exp(power);
        double ea = 16.0 * u * (1.0 + 0.5 * (fabs(qa) + fabs(qc)) + fabs(qb));
        if (a > 0.99) {
            if (a > 0.99 * (1.0 + ea)) ea = 2.0 * u;
            a = 0.99;
        }
        double ma = fabs(255.0 * a - 1.0) / ea;
        if (ma < m_alpha) m_alpha = ma;
        if (a < 1.0 / 255.0) continue;
        double Tn = T * (1.0 - a);
        double eTn = eT + 0.5 * ea * a / (1.0 - a) + u;
        double mt = fabs(Tn * 1e4 - 1.0) / eTn;
        if (mt < m_T) m_T = mt;
        if (Tn < 1e-4) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += a * T * rgb[ch * n + i];
        T = Tn;
        eT = eTn;
        last = j + 1;
    }
    for (int ch = 0; ch < 3; ++ch) out5[ch] = C[ch] + T * bg[ch];
    out5[3] = T;
    out5[4] = (double)last;
    margins2[0] = m_alpha;
    margins2[1] = m_T;
}

/* Full image along the tile lists: values sorted per tile, ranges[t][2].
 * out_rgb[3][H][W], out_T[H][W], out_nc[H][W], out_margin[2][H][W]. */
void or_composite(int width, int height, const uint64_t* ranges, const uint32_t* values, int64_t n,
                  const double* mean2d, const double* conic, const double* opacity, const double* rgb,
                  const double* bg3, double* out_rgb, double* out_T, int32_t* out_nc, double* out_margin)
{
    int tiles_x = (width + TILE - 1) / TILE;
    int64_t P = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 4)
    for (int py = 0; py < height; ++py)
        for (int px = 0; px < width; ++px) {
            int64_t t = (int64_t)(py / TILE) * tiles_x + px / TILE;
            uint64_t s = ranges[2 * t], e = ranges[2 * t + 1];
            double o[5], m[2];
            composite_pixel(px, py, values + s, (int64_t)(e - s), n, mean2d, conic, opacity, rgb, bg3, o, m);
            int64_t p = (int64_t)py * width + px;
            for (int ch = 0; ch < 3; ++ch) out_rgb[ch * P + p] = o[ch];
            out_T[p] = o[3];
            out_nc[p] = (int32_t)o[4];
            out_margin[p] = m[0];
            out_margin[P + p] = m[1];
        }
}

/* Selected pixels (px[k], py[k]) along one shared list (all in one tile). */
void or_composite_pixels(int64_t count, const int32_t* px, const int32_t* py, const uint32_t* list,
                         int64_t len, int64_t n, const double* mean2d, const double* conic,
                         const double* opacity, const double* rgb, const double* bg3,
                         double* out5, double* out_margin2)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k)
        composite_pixel(px[k], py[k], list, len, n, mean2d, conic, opacity, rgb, bg3,
                        out5 + 5 * k, out_margin2 + 2 * k);
}

/* Selected tiles of the image, each one on its own: the tile's list (every
 * Gaussian whose rectangle holds the tile, ordered by (depth_bits, index),
 * the list of or_tile_list) and every pixel of the tile composited along it
 * (composite_pixel), tiles in parallel.  The Gaussians of each tile row are
 * gathered once, in index order, so a tile's list comes from its row's
 * candidates instead of all n.  tiles[count] are tile indices (row-major);
 * only their pixels of out_rgb[3][H][W], out_T, out_nc and out_margin[2][H][W]
 * are written. */
void or_render_tiles(int width, int height, int64_t n, const int32_t* rect, const uint32_t* tiles_touched,
                     const uint32_t* depth_bits, const double* mean2d, const double* conic, const double* opacity,
                     const double* rgb, const double* bg3, const int64_t* tiles, int64_t count, double* out_rgb,
                     double* out_T, int32_t* out_nc, double* out_margin)
{
    int tiles_x = (width + TILE - 1) / TILE, tiles_y = (height + TILE - 1) / TILE;
    int64_t P = (int64_t)width * height;
    /* the tile rows the selection needs, and their candidates */
    char* need = (char*)calloc((size_t)tiles_y, 1);
    for (int64_t k = 0; k < count; ++k) need[tiles[k] / tiles_x] = 1;
    int64_t* row_count = (int64_t*)calloc((size_t)tiles_y + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (tiles_touched[i] == 0) continue;
        for (int32_t ty = rect[n + i]; ty < rect[3 * n + i]; ++ty)
            if (need[ty]) ++row_count[ty + 1];
    }
    for (int ty = 0; ty < tiles_y; ++ty) row_count[ty + 1] += row_count[ty];
    uint32_t* cand = (uint32_t*)malloc((size_t)(row_count[tiles_y] > 0 ? row_count[tiles_y] : 1) * sizeof(uint32_t));
    int64_t* fill = (int64_t*)malloc((size_t)tiles_y * sizeof(int64_t));
    for (int ty = 0; ty < tiles_y; ++ty) fill[ty] = row_count[ty];
    for (int64_t i = 0; i < n; ++i) {
        if (tiles_touched[i] == 0) continue;
        for (int32_t ty = rect[n + i]; ty < rect[3 * n + i]; ++ty)
            if (need[ty]) cand[fill[ty]++] = (uint32_t)i;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k) {
        int64_t tile = tiles[k];
        int32_t tx = (int32_t)(tile % tiles_x), ty = (int32_t)(tile / tiles_x);
        int64_t c0 = row_count[ty], c1 = row_count[ty + 1], m = 0;
        depth_entry_t* e = (depth_entry_t*)malloc((size_t)(c1 > c0 ? c1 - c0 : 1) * sizeof(depth_entry_t));
        for (int64_t c = c0; c < c1; ++c) {
            uint32_t i = cand[c];
            if (tx < rect[i] || tx >= rect[2 * n + i]) continue;
            e[m].bits = depth_bits[i];
            e[m].index = i;
            ++m;
        }
        qsort(e, (size_t)m, sizeof(depth_entry_t), cmp_depth_entry);
        uint32_t* list = (uint32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint32_t));
        for (int64_t j = 0; j < m; ++j) list[j] = e[j].index;
        for (int py = ty * TILE; py < ty * TILE + TILE && py < height; ++py)
            for (int px = tx * TILE; px < tx * TILE + TILE && px < width; ++px) {
                double o[5], mg[2];
                composite_pixel(px, py, list, m, n, mean2d, conic, opacity, rgb, bg3, o, mg);
                int64_t p = (int64_t)py * width + px;
                for (int ch = 0; ch < 3; ++ch) out_rgb[ch * P + p] = o[ch];
                out_T[p] = o[3];
                out_nc[p] = (int32_t)o[4];
                out_margin[p] = mg[0];
                out_margin[P + p] = mg[1];
            }
        free(list);
        free(e);
    }
    free(fill);
    free(cand);
    free(row_count);
    free(need);
}

typedef struct { double depth; uint32_t index; } brute_entry_t;

static int cmp_brute(const void* a, const void* b)
{
    const brute_entry_t* p = (const brute_entry_t*)a;
    const brute_entry_t* q = (const brute_entry_t*)b;
    if (p->depth != q->depth) return p->depth < q->depth ? -1 : 1;
    if (p->index != q->index) return p->index < q->index ? -1 : 1;
    return 0;
}

/* Brute force: every pixel composites every Gaussian that survives the
 * geometric culls (in front of the near plane, finite, positive-definite 2D
 * covariance), ordered by (FP64 depth, index), with no tiles and no bounding
 * square.  geom_ok[n] marks those survivors (radius_margin finite). */
void or_bruteforce(int width, int height, int64_t n, const double* radius_margin,
                   const double* depth, const double* mean2d, const double* conic,
                   const double* opacity, const double* rgb, const double* bg3,
                   double* out_rgb, double* out_T, int32_t* out_nc)
{
    int64_t m = 0;
    brute_entry_t* e = (brute_entry_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(brute_entry_t));
    for (int64_t i = 0; i < n; ++i)
        if (isfinite(radius_margin[i])) { e[m].depth = depth[i]; e[m].index = (uint32_t)i; ++m; }
    qsort(e, (size_t)m, sizeof(brute_entry_t), cmp_brute);
    uint32_t* list = (uint32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint32_t));
    for (int64_t j = 0; j < m; ++j) list[j] = e[j].index;
    int64_t P = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 4)
    for (int py = 0; py < height; ++py)
        for (int px = 0; px < width; ++px) {
            double o[5], mg[2];
            composite_pixel(px, py, list, m, n, mean2d, conic, opacity, rgb, bg3, o, mg);
            int64_t p = (int64_t)py * width + px;
            for (int ch = 0; ch < 3; ++ch) out_rgb[ch * P + p] = o[ch];
            out_T[p] = o[3];
            out_nc[p] = (int32_t)o[4];
        }
    free(list);
    free(e);
}

/* Threads the parallel loops use from now on (timing at one thread and at
 * all cores); n <= 0 restores the default. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
