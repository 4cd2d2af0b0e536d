/*
 * CPU oracle for the factorized shading bake of Factorized Inverse Path
 * Tracing (Wu, Zhu et al., ICCV 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code with the
 * GPU library and the GPU library never calls it.
 *
 * Plain, slow and obviously correct: every quantity is computed in double
 * precision from the single-precision inputs (promoted exactly), every ray
 * is tested against every triangle (no acceleration structure), and sums run
 * in sample order.
 *
 * What it computes, with the paper's equations:
 *   - camera ray through each pixel centre -> closest hit x, face normal n
 *     facing the viewer, outgoing direction wo = -dir (the (x, wo) pairs of
 *     Eq. 2);
 *   - the shading integrals of Eq. 6 with the Fresnel split of Eq. 7,
 *     estimated by importance-sampled Monte Carlo with the stage-1 radiance
 *     query of Eq. 9 (incident radiance = radiance cache + per-triangle
 *     emission at the first hit, zero on a miss); the cache is per
 *     triangle, per vertex (barycentric blend), or, as Sec. 4.2 builds it,
 *     a voxel grid read at the voxel that contains the hit point (nearest
 *     voxel; voxel (i, j, k) of an R^3 grid over [lo, hi] holds the points
 *     with floor((x - lo) R / (hi - lo)) = (i, j, k), clamped to the grid):
 *       Ld       = mean over cosine-distributed wi of R
 *       Ls0_k    = mean over GGX-sampled half vectors of R * F0 * w
 *       Ls1_k    = mean over GGX-sampled half vectors of R * F1 * w
 *     with w = G * (wo.m) / ((n.wo)(n.m)), i.e. F*D*G/(4 n.wo) divided by
 *     the density of wi when m is drawn from D(m)(n.m);
 *   - D is GGX (Walter et al. 2007), G the separable Smith product of
 *     Walter's GGX G1, F1 = (1 - wi.m)^5 and F0 = 1 - F1 (Schlick, Eq. 7);
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (point lo, point hi, lobe, sample);
 *   - for every sample whose ray passes close enough to a triangle edge or
 *     to a second surface that single-precision arithmetic may legitimately
 *     pick another result, the envelope [lo, hi] of every possible outcome.
 *
 * Readings where the paper is silent (all shared with the GPU path by
 * specification, not by code): alpha = sigma^2; geometric face normal
 * flipped toward wo; ray origin x + eps*n; samples below the horizon count
 * as zero; misses return zero; exact distance ties go to the lower triangle
 * index; orthonormal frame of Duff et al. 2017 with the sign taken as
 * (n.z >= 0 ? 1 : -1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, from its published definition: ten rounds of two 32x32   */
/* multiplies (constants 0xD2511F53, 0xCD9E8D57) with a Weyl key schedule  */
/* (0x9E3779B9, 0xBB67AE85) applied between rounds.                        */
/* ---------------------------------------------------------------------- */
static void philox(const uint32_t c_in[4], const uint32_t k_in[2], uint32_t out[4])
{
    uint32_t x0 = c_in[0], x1 = c_in[1], x2 = c_in[2], x3 = c_in[3];
    uint32_t k0 = k_in[0], k1 = k_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) philox(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Cell (x, y) of a 2^k x 2^k grid at distance d along the Hilbert curve that
 * starts in cell (0, 0) and ends in cell (2^k - 1, 0): the quadrant of each
 * level is read from two bits of d, finest level first, and the partial
 * cell is reflected and transposed as the curve's orientation requires
 * (the curve of Hilbert 1891, in its common iterative form). */
static void hilbert_cell(int k, uint32_t d, uint32_t* x, uint32_t* y)
{
    uint32_t cx = 0, cy = 0;
    for (uint32_t side = 1; side < (1u << k); side *= 2) {
        const uint32_t qx = (d >> 1) & 1u;
        const uint32_t qy = (d ^ qx) & 1u;
        if (qy == 0) {
            if (qx == 1) {
                cx = side - 1 - cx;
                cy = side - 1 - cy;
            }
            const uint32_t t = cx;
            cx = cy;
            cy = t;
        }
        cx += side * qx;
        cy += side * qy;
        d >>= 2;
    }
    *x = cx;
    *y = cy;
}

/* The two uniforms of sample s of a lobe's n samples, stratified along a
 * curve through the unit square.  The 32-bit line is cut into n segments
 * of width W = floor(2^32 / n); sample s takes the point
 * U = s W + floor(u0 W / 2^32) of its own segment (u the Philox block of the
 * counter (p low, p high, lobe, s)).  The top four bits of U pick a cell of
 * the 4 x 4 grid along the Hilbert curve; the other 28 bits, read as a
 * Morton code (bit 2i to the column, bit 2i + 1 to the row), place the
 * point inside that cell on a 2^14 x 2^14 grid.  A point inside the finest
 * cell comes from the top bytes of u1 and u2, so each coordinate has 24
 * bits: xi1 = (2^8 X + (u1 >> 24)) / 2^24, xi2 = (2^8 Y + (u2 >> 24)) / 2^24.
 * The segments tile [0, nW), all but less than n / 2^32 of the square, so
 * the estimate is stratified and unbiased up to that sliver. */
static void sample_uniforms(uint64_t seed, int64_t p, int lobe, int s, int n,
                            double* xi1, double* xi2)
{
    uint32_t c[4] = {(uint32_t)(uint64_t)p, (uint32_t)((uint64_t)p >> 32),
                     (uint32_t)lobe, (uint32_t)s};
    uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t u[4];
    philox(c, k, u);
    const uint64_t W = ((uint64_t)1 << 32) / (uint64_t)n;
    const uint64_t U = (uint64_t)s * W + (((uint64_t)u[0] * W) >> 32);
    uint32_t cx, cy;
    hilbert_cell(2, (uint32_t)(U >> 28), &cx, &cy);
    uint32_t X = cx << 14, Y = cy << 14;
    for (int i = 0; i < 14; ++i) {
        X |= (uint32_t)((U >> (2 * i)) & 1u) << i;
        Y |= (uint32_t)((U >> (2 * i + 1)) & 1u) << i;
    }
    *xi1 = ((double)X * 256.0 + (double)(u[1] >> 24)) / 16777216.0;
    *xi2 = ((double)Y * 256.0 + (double)(u[2] >> 24)) / 16777216.0;
}

/* The uniforms of samples s[i] of n[i] for lobe lobe[i] of point p[i]. */
void orc_lobe_uniforms(uint64_t seed, const int64_t* p, const int32_t* lobe, const int32_t* s,
                       const int32_t* n, int64_t count, double* xi1, double* xi2)
{
    for (int64_t i = 0; i < count; ++i)
        sample_uniforms(seed, p[i], lobe[i], s[i], n[i], xi1 + i, xi2 + i);
}

/* ---------------------------------------------------------------------- */
/* small vector helpers                                                    */
/* ---------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* Orthonormal frame around a unit normal (Duff et al., JCGT 6(1), 2017). */
void orc_frame(const double n[3], double t[3], double b[3])
{
    double s = (n[2] >= 0.0) ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double c = n[0] * n[1] * a;
    t[0] = 1.0 + s * n[0] * n[0] * a;
    t[1] = s * c;
    t[2] = -s * n[0];
    b[0] = c;
    b[1] = s + n[1] * n[1] * a;
    b[2] = -n[1];
}

static void to_world(const double t[3], const double b[3], const double n[3],
                     const double l[3], double w[3])
{
    for (int i = 0; i < 3; ++i) w[i] = t[i] * l[0] + b[i] * l[1] + n[i] * l[2];
}

/* Cosine-weighted hemisphere direction, local frame (z = normal). */
void orc_sample_cosine(double xi1, double xi2, double out[3])
{
    double r = sqrt(xi1), phi = 2.0 * ORC_PI * xi2;
    out[0] = r * cos(phi);
    out[1] = r * sin(phi);
    out[2] = sqrt(1.0 - xi1);
}

/* GGX half vector with density D(m)(n.m) (Walter et al. 2007, Eqs. 35-36):
 * tan^2(theta_m) = alpha^2 xi1 / (1 - xi1), phi_m = 2 pi xi2. */
void orc_sample_ggx(double alpha, double xi1, double xi2, double out[3])
{
    double tan2 = alpha * alpha * xi1 / (1.0 - xi1);
    double cos_t = 1.0 / sqrt(1.0 + tan2);
    double sin_t = sqrt(fmax(0.0, 1.0 - cos_t * cos_t));
    double phi = 2.0 * ORC_PI * xi2;
    out[0] = sin_t * cos(phi);
    out[1] = sin_t * sin(phi);
    out[2] = cos_t;
}

/* GGX normal distribution D(m) for cos(theta_m) = n.m > 0. */
double orc_ggx_D(double alpha, double cos_m)
{
    if (cos_m <= 0.0) return 0.0;
    double a2 = alpha * alpha;
    double c2 = cos_m * cos_m;
    double tan2 = (1.0 - c2) / c2;
    double d = c2 * c2 * (a2 + tan2) * (a2 + tan2);
    return a2 / (ORC_PI * d);
}

/* Smith G1 for GGX (Walter et al. 2007): 2 / (1 + sqrt(1 + alpha^2 tan^2)),
 * valid when v.m and v.n have the same sign; cos_v = n.v > 0. */
double orc_ggx_G1(double alpha, double cos_v)
{
    if (cos_v <= 0.0) return 0.0;
    double c2 = cos_v * cos_v;
    double tan2 = (1.0 - c2) / c2;
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

/* ---------------------------------------------------------------------- */
/* scene                                                                   */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t V, T;
    double* v0;    /* [T][3] */
    double* e1;    /* [T][3] v1 - v0 */
    double* e2;    /* [T][3] v2 - v0 */
    double* h;     /* [T][3] distance from vertex i to its opposite edge */
    double* slack; /* [T] barycentric slack covering the largest tolerance */
    double* emin;  /* [T] 1e-14 * |e1| |e2| (parallel-ray threshold) */
    int32_t* tri;  /* [T][3] */
    int cache_kind;            /* 0: per triangle [3][T], 1: per vertex [3][V],
                                  2: voxel grid [3][R^3], x fastest */
    double* cache;             /* [3][n] */
    int vox_res;               /* R */
    double vox_lo[3], vox_hi[3];
    double* emission;          /* [3][T] */
    double tol_rel;            /* ambiguity tolerance, relative to 1 + t */
} scene_t;

void* orc_scene_new(const float* verts, int64_t V, const int32_t* tris, int64_t T,
                    int cache_kind, const float* cache, const float* emission,
                    double tol_rel, double max_t)
{
    scene_t* S = (scene_t*)calloc(1, sizeof(scene_t));
    S->V = V;
    S->T = T;
    S->v0 = (double*)malloc(sizeof(double) * 3 * T);
    S->e1 = (double*)malloc(sizeof(double) * 3 * T);
    S->e2 = (double*)malloc(sizeof(double) * 3 * T);
    S->h = (double*)malloc(sizeof(double) * 3 * T);
    S->slack = (double*)malloc(sizeof(double) * T);
    S->emin = (double*)malloc(sizeof(double) * T);
    S->tri = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    S->cache_kind = cache_kind;
    int64_t nc = cache_kind ? V : T;
    S->cache = (double*)malloc(sizeof(double) * 3 * nc);
    S->emission = (double*)malloc(sizeof(double) * 3 * T);
    S->tol_rel = tol_rel;
    for (int64_t i = 0; i < 3 * nc; ++i) S->cache[i] = (double)cache[i];
    for (int64_t i = 0; i < 3 * T; ++i) S->emission[i] = (double)emission[i];
    for (int64_t f = 0; f < T; ++f) {
        double p[3][3];
        for (int k = 0; k < 3; ++k) {
            int32_t vi = tris[3 * f + k];
            S->tri[3 * f + k] = vi;
            for (int c = 0; c < 3; ++c) p[k][c] = (double)verts[3 * (int64_t)vi + c];
        }
        for (int c = 0; c < 3; ++c) {
            S->v0[3 * f + c] = p[0][c];
            S->e1[3 * f + c] = p[1][c] - p[0][c];
            S->e2[3 * f + c] = p[2][c] - p[0][c];
        }
        double cr[3], e12[3];
        cross3(S->e1 + 3 * f, S->e2 + 3 * f, cr);
        double area2 = norm3(cr);
        for (int c = 0; c < 3; ++c) e12[c] = p[2][c] - p[1][c];
        double l_e1 = norm3(S->e1 + 3 * f), l_e2 = norm3(S->e2 + 3 * f), l_12 = norm3(e12);
        /* barycentric weight of vertex 0 / 1 / 2 times these heights gives
         * the distance to the opposite edge */
        S->h[3 * f + 0] = l_12 > 0 ? area2 / l_12 : 0.0;
        S->h[3 * f + 1] = l_e2 > 0 ? area2 / l_e2 : 0.0;
        S->h[3 * f + 2] = l_e1 > 0 ? area2 / l_e1 : 0.0;
        double hmin = fmin(S->h[3 * f], fmin(S->h[3 * f + 1], S->h[3 * f + 2]));
        S->slack[f] = hmin > 0 ? 2.0 * tol_rel * (1.0 + max_t) / hmin : 1e300;
        S->emin[f] = 1e-14 * l_e1 * l_e2;
    }
    return S;
}

/* Switch the scene's cache to a voxel grid: cache [3][res^3] (x fastest)
 * over the box [lo, hi]. */
int orc_scene_set_voxel(void* sp, const float* cache, int res, const double* lo, const double* hi)
{
    scene_t* S = (scene_t*)sp;
    if (res < 1) return -1;
    for (int a = 0; a < 3; ++a)
        if (!(hi[a] > lo[a])) return -1;
    int64_t nv = (int64_t)res * res * res;
    double* c = (double*)malloc(sizeof(double) * 3 * nv);
    if (!c) return -1;
    for (int64_t i = 0; i < 3 * nv; ++i) c[i] = (double)cache[i];
    free(S->cache);
    S->cache = c;
    S->cache_kind = 2;
    S->vox_res = res;
    for (int a = 0; a < 3; ++a) {
        S->vox_lo[a] = lo[a];
        S->vox_hi[a] = hi[a];
    }
    return 0;
}

void orc_scene_free(void* p)
{
    scene_t* S = (scene_t*)p;
    if (!S) return;
    free(S->v0); free(S->e1); free(S->e2); free(S->h); free(S->slack);
    free(S->emin); free(S->tri); free(S->cache); free(S->emission);
    free(S);
}

/* ---------------------------------------------------------------------- */
/* brute-force ray casting                                                 */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t tri;
    double t, b1, b2;
} hit_t;

#define MAX_CAND 256
/* Returned by every entry point that casts rays when some ray met more
 * candidate outcomes than MAX_CAND: its envelope would be incomplete, so the
 * result is refused rather than truncated. */
#define ORC_EOVERFLOW (-2)

typedef struct {
    hit_t nominal;          /* nearest exact hit, tri = -1 on a miss */
    int n_cand;             /* outcomes single precision may also produce */
    hit_t cand[MAX_CAND];   /* tri = -1 entry stands for "miss" */
    int overflow;
} cast_t;

/* Moller-Trumbore against every triangle.  The exact hit test is
 * b1 >= 0, b2 >= 0, b1 + b2 <= 1, t > 0; the nearest such t wins, ties to
 * the lower index.  Besides it, every triangle whose hit point lies within
 * tol_rel * (1 + t) of one of its edges (inside or outside), or whose plane
 * crosses the ray within tol_rel of its origin, is "uncertain"; the
 * possible outcomes are the nearest certain hit (or a miss when there is
 * none) and every uncertain or certain hit no farther than that. */
static void cast(const scene_t* S, const double o[3], const double d[3], cast_t* out)
{
    hit_t cert[MAX_CAND], unc[MAX_CAND];
    int nc = 0, nu = 0;
    out->overflow = 0;
    out->nominal.tri = -1;
    out->nominal.t = INFINITY;
    out->nominal.b1 = out->nominal.b2 = 0.0;
    double tA = INFINITY;
    hit_t fallback = {-1, INFINITY, 0.0, 0.0};
    for (int64_t f = 0; f < S->T; ++f) {
        const double* e1 = S->e1 + 3 * f;
        const double* e2 = S->e2 + 3 * f;
        double pv[3];
        cross3(d, e2, pv);
        double det = dot3(e1, pv);
        if (fabs(det) <= S->emin[f]) continue;
        double inv = 1.0 / det;
        double sv[3] = {o[0] - S->v0[3 * f], o[1] - S->v0[3 * f + 1], o[2] - S->v0[3 * f + 2]};
        double b1 = dot3(sv, pv) * inv;
        double sl = S->slack[f];
        if (b1 < -sl || b1 > 1.0 + sl) continue;
        double qv[3];
        cross3(sv, e1, qv);
        double b2 = dot3(d, qv) * inv;
        if (b2 < -sl || b1 + b2 > 1.0 + sl) continue;
        double t = dot3(e2, qv) * inv;
        /* a plane through (or within the band of) the ray origin may be hit
         * or missed by rounding, like a nearby edge */
        if (t <= -S->tol_rel) continue;
        int near_origin = (t <= S->tol_rel);
        double b0 = 1.0 - b1 - b2;
        int inside = (b0 >= 0.0 && b1 >= 0.0 && b2 >= 0.0);
        if (inside && t > 0.0 &&
            (t < out->nominal.t || (t == out->nominal.t && f < out->nominal.tri))) {
            out->nominal.tri = (int32_t)f;
            out->nominal.t = t;
            out->nominal.b1 = b1;
            out->nominal.b2 = b2;
        }
        double m0 = b0 * S->h[3 * f], m1 = b1 * S->h[3 * f + 1], m2 = b2 * S->h[3 * f + 2];
        double margin = fmin(m0, fmin(m1, m2));
        double dtol = S->tol_rel * (1.0 + t);
        hit_t hh = {(int32_t)f, t, b1, b2};
        if (!inside && t > 0.0 && margin >= -dtol &&
            (t < fallback.t || (t == fallback.t && f < fallback.tri)))
            fallback = hh;
        if (margin > dtol && !near_origin) {
            if (nc < MAX_CAND) cert[nc++] = hh; else out->overflow = 1;
            if (t < tA) tA = t;
        } else if (margin >= -dtol) {
            if (nu < MAX_CAND) unc[nu++] = hh; else out->overflow = 1;
        }
    }
    /* A ray that passes through a shared edge can fail the exact test on
     * both triangles by rounding alone; a mesh without gaps is hit there, so
     * with no exact hit the nearest hit within the tolerance band stands. */
    if (out->nominal.tri < 0 && fallback.tri >= 0) {
        out->nominal = fallback;
        double w0 = fmax(1.0 - fallback.b1 - fallback.b2, 0.0);
        double w1 = fmax(fallback.b1, 0.0), w2 = fmax(fallback.b2, 0.0);
        double sum = w0 + w1 + w2;
        out->nominal.b1 = w1 / sum;
        out->nominal.b2 = w2 / sum;
    }
    double lim = isinf(tA) ? INFINITY : tA + S->tol_rel * (1.0 + tA);
    int n = 0;
    for (int i = 0; i < nc; ++i)
        if (cert[i].t <= lim && n < MAX_CAND) out->cand[n++] = cert[i];
    for (int i = 0; i < nu; ++i)
        if (unc[i].t <= lim && n < MAX_CAND) out->cand[n++] = unc[i];
    if (isinf(tA) && n < MAX_CAND) {
        hit_t miss = {-1, INFINITY, 0.0, 0.0};
        out->cand[n++] = miss;
    }
    out->n_cand = n;
}

/* Hit point of a hit: v0 + b1 e1 + b2 e2. */
static void hit_point(const scene_t* S, const hit_t* h, double x[3])
{
    int64_t f = h->tri;
    for (int a = 0; a < 3; ++a)
        x[a] = S->v0[3 * f + a] + h->b1 * S->e1[3 * f + a] + h->b2 * S->e2[3 * f + a];
}

/* Voxel coordinate of x along axis a (before flooring). */
static double voxel_coord(const scene_t* S, const double x[3], int a)
{
    return (x[a] - S->vox_lo[a]) * S->vox_res / (S->vox_hi[a] - S->vox_lo[a]);
}

static int voxel_clamp(const scene_t* S, double u)
{
    double i = floor(u);
    if (i < 0.0) return 0;
    if (i > S->vox_res - 1) return S->vox_res - 1;
    return (int)i;
}

static int64_t voxel_linear(const scene_t* S, int i, int j, int k)
{
    return ((int64_t)k * S->vox_res + j) * S->vox_res + i;
}

/* Radiance leaving the hit toward the ray origin: radiance cache (per
 * triangle, per vertex interpolated with barycentric weights, or the voxel
 * that contains the hit point) plus the triangle's emission; zero on a miss
 * (Eq. 9 with per-triangle emission). */
static void radiance(const scene_t* S, const hit_t* h, int clamp, double R[3])
{
    if (h->tri < 0) {
        R[0] = R[1] = R[2] = 0.0;
        return;
    }
    int64_t f = h->tri;
    for (int c = 0; c < 3; ++c) R[c] = S->emission[c * S->T + f];
    if (S->cache_kind == 2) {
        double x[3];
        hit_point(S, h, x);
        int64_t v = voxel_linear(S, voxel_clamp(S, voxel_coord(S, x, 0)),
                                 voxel_clamp(S, voxel_coord(S, x, 1)),
                                 voxel_clamp(S, voxel_coord(S, x, 2)));
        int64_t nv = (int64_t)S->vox_res * S->vox_res * S->vox_res;
        for (int c = 0; c < 3; ++c) R[c] += S->cache[c * nv + v];
    } else if (S->cache_kind == 0) {
        for (int c = 0; c < 3; ++c) R[c] += S->cache[c * S->T + f];
    } else {
        double w1 = h->b1, w2 = h->b2, w0 = 1.0 - w1 - w2;
        if (clamp) {
            w0 = fmax(w0, 0.0); w1 = fmax(w1, 0.0); w2 = fmax(w2, 0.0);
            double s = w0 + w1 + w2;
            w0 /= s; w1 /= s; w2 /= s;
        }
        const int32_t* vi = S->tri + 3 * f;
        for (int c = 0; c < 3; ++c)
            R[c] += w0 * S->cache[c * S->V + vi[0]] + w1 * S->cache[c * S->V + vi[1]]
                  + w2 * S->cache[c * S->V + vi[2]];
    }
}

/* With a voxel cache: widen [Rmin, Rmax] by the radiance of every voxel
 * whose face lies within the rounding band of the hit point (single
 * precision may place the point in either voxel).  Returns 1 if it did. */
static int voxel_ties(const scene_t* S, const hit_t* h, double Rmin[3], double Rmax[3])
{
    if (S->cache_kind != 2 || h->tri < 0) return 0;
    double x[3];
    hit_point(S, h, x);
    double mag = fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
    int lo_i[3], hi_i[3], wide = 0;
    for (int a = 0; a < 3; ++a) {
        double band = S->tol_rel * (1.0 + h->t + mag) * S->vox_res / (S->vox_hi[a] - S->vox_lo[a]);
        double u = voxel_coord(S, x, a);
        lo_i[a] = voxel_clamp(S, u - band);
        hi_i[a] = voxel_clamp(S, u + band);
        if (hi_i[a] != lo_i[a]) wide = 1;
    }
    if (!wide) return 0;
    int64_t nv = (int64_t)S->vox_res * S->vox_res * S->vox_res;
    int64_t f = h->tri;
    for (int k = lo_i[2]; k <= hi_i[2]; ++k)
        for (int j = lo_i[1]; j <= hi_i[1]; ++j)
            for (int i = lo_i[0]; i <= hi_i[0]; ++i) {
                int64_t v = voxel_linear(S, i, j, k);
                for (int c = 0; c < 3; ++c) {
                    double r = S->emission[c * S->T + f] + S->cache[c * nv + v];
                    Rmin[c] = fmin(Rmin[c], r);
                    Rmax[c] = fmax(Rmax[c], r);
                }
            }
    return 1;
}

/* Nominal radiance plus its per-channel minimum and maximum over every
 * outcome single precision may produce. */
static int radiance_envelope(const scene_t* S, const cast_t* h, double R[3],
                             double Rmin[3], double Rmax[3])
{
    radiance(S, &h->nominal, 0, R);
    for (int c = 0; c < 3; ++c) Rmin[c] = Rmax[c] = R[c];
    int ambiguous = voxel_ties(S, &h->nominal, Rmin, Rmax);
    for (int i = 0; i < h->n_cand; ++i) {
        double r[3];
        radiance(S, &h->cand[i], 1, r);
        for (int c = 0; c < 3; ++c) {
            Rmin[c] = fmin(Rmin[c], r[c]);
            Rmax[c] = fmax(Rmax[c], r[c]);
        }
        ambiguous |= voxel_ties(S, &h->cand[i], Rmin, Rmax);
    }
    if (h->n_cand > 1 || (h->n_cand == 1 && h->cand[0].tri != h->nominal.tri)) ambiguous = 1;
    return ambiguous;
}

/* Rays cast one by one (test hook): nominal hit, barycentrics, outcome count. */
int orc_cast(void* sp, const double* o, const double* d, int64_t n, int32_t* tri,
             double* t, double* b, int32_t* n_cand)
{
    const scene_t* S = (const scene_t*)sp;
    cast_t* h = (cast_t*)malloc(sizeof(cast_t));
    int overflow = 0;
    for (int64_t i = 0; i < n; ++i) {
        cast(S, o + 3 * i, d + 3 * i, h);
        overflow |= h->overflow;
        tri[i] = h->nominal.tri;
        t[i] = h->nominal.t;
        b[2 * i] = h->nominal.b1;
        b[2 * i + 1] = h->nominal.b2;
        n_cand[i] = h->n_cand;
    }
    free(h);
    return overflow ? ORC_EOVERFLOW : 0;
}

/* Radiance arriving along each ray (test hook): nominal hit, cache plus
 * emission, zero on a miss. */
int orc_trace_radiance(void* sp, const double* o, const double* d, int64_t n, double* R)
{
    const scene_t* S = (const scene_t*)sp;
    cast_t* h = (cast_t*)malloc(sizeof(cast_t));
    int overflow = 0;
    for (int64_t i = 0; i < n; ++i) {
        cast(S, o + 3 * i, d + 3 * i, h);
        overflow |= h->overflow;
        radiance(S, &h->nominal, 0, R + 3 * i);
    }
    free(h);
    return overflow ? ORC_EOVERFLOW : 0;
}

/* ---------------------------------------------------------------------- */
/* shading points from pinhole cameras                                      */
/* ---------------------------------------------------------------------- */
/* Camera row: pos(3) fwd(3) up(3) vfov_deg; size: width, height.  Pixel
 * (i, j) of camera c has global index offset(c) + j * width + i; its ray
 * passes through the pixel centre. */
static void camera_ray(const float* cam, int W, int H, int i, int j, double o[3], double d[3])
{
    double f[3] = {cam[3], cam[4], cam[5]}, up[3] = {cam[6], cam[7], cam[8]};
    double fl = norm3(f);
    for (int k = 0; k < 3; ++k) f[k] /= fl;
    double r[3], u[3];
    cross3(f, up, r);
    double rl = norm3(r);
    for (int k = 0; k < 3; ++k) r[k] /= rl;
    cross3(r, f, u);
    double th = tan(0.5 * (double)cam[9] * ORC_PI / 180.0);
    double aspect = (double)W / (double)H;
    double sx = (2.0 * (i + 0.5) / W - 1.0) * th * aspect;
    double sy = (1.0 - 2.0 * (j + 0.5) / H) * th;
    for (int k = 0; k < 3; ++k) d[k] = f[k] + sx * r[k] + sy * u[k];
    double dl = norm3(d);
    for (int k = 0; k < 3; ++k) {
        d[k] /= dl;
        o[k] = cam[k];
    }
}

/* out: [9][n] px py pz nx ny nz ox oy oz; tri[n]; ambig[n] = outcome count. */
int orc_primary(void* sp, const float* cams, const int32_t* sizes, int n_cams,
                const int64_t* idx, int64_t n, double* out, int32_t* tri_out,
                int32_t* ambig, int n_threads)
{
    const scene_t* S = (const scene_t*)sp;
    int64_t* offs = (int64_t*)malloc(sizeof(int64_t) * (n_cams + 1));
    offs[0] = 0;
    for (int c = 0; c < n_cams; ++c) offs[c + 1] = offs[c] + (int64_t)sizes[2 * c] * sizes[2 * c + 1];
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int bad = 0, overflow = 0;
#pragma omp parallel reduction(| : overflow)
    {
        cast_t* h = (cast_t*)malloc(sizeof(cast_t));
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < n; ++q) {
            int64_t p = idx[q];
            int c = 0;
            while (c < n_cams && p >= offs[c + 1]) ++c;
            if (c >= n_cams || p < 0) {
                bad = 1;
                continue;
            }
            int W = sizes[2 * c], H = sizes[2 * c + 1];
            int64_t local = p - offs[c];
            int i = (int)(local % W), j = (int)(local / W);
            double o[3], d[3];
            camera_ray(cams + 10 * c, W, H, i, j, o, d);
            cast(S, o, d, h);
            overflow |= h->overflow;
            ambig[q] = h->n_cand;
            tri_out[q] = h->nominal.tri;
            if (h->nominal.tri < 0) {
                for (int k = 0; k < 9; ++k) out[k * n + q] = 0.0;
                continue;
            }
            int64_t f = h->nominal.tri;
            double nn[3];
            cross3(S->e1 + 3 * f, S->e2 + 3 * f, nn);
            double l = norm3(nn);
            for (int k = 0; k < 3; ++k) nn[k] /= l;
            if (dot3(nn, d) > 0.0)
                for (int k = 0; k < 3; ++k) nn[k] = -nn[k];
            for (int k = 0; k < 3; ++k) {
                out[k * n + q] = o[k] + h->nominal.t * d[k];
                out[(3 + k) * n + q] = nn[k];
                out[(6 + k) * n + q] = -d[k];
            }
        }
        free(h);
    }
    free(offs);
    return bad ? -1 : overflow ? ORC_EOVERFLOW : 0;
}

/* ---------------------------------------------------------------------- */
/* the bake                                                                */
/* ---------------------------------------------------------------------- */
#define ORC_WEAK_FURNACE 1  /* test flag: R = 1 without casting, G = G1(wo),
                               no horizon rejection */

/* Specular sample weight for one half vector m (world), given n, wo and
 * cos_o = n.wo > 0.  Returns 0 for samples outside the domain of Eq. 6.
 * w = G (wo.m) / ((n.wo)(n.m)); F1 = (1 - wi.m)^5. */
static double spec_weight(double alpha, const double n[3], const double wo[3],
                          double cos_o, const double m[3], double wi[3],
                          double* F1, int flags)
{
    double om = dot3(wo, m);
    if (om <= 0.0) return 0.0;
    for (int k = 0; k < 3; ++k) wi[k] = 2.0 * om * m[k] - wo[k];
    double ci = dot3(n, wi);
    double cm = dot3(n, m);
    if (cm <= 0.0) return 0.0;
    double G;
    if (flags & ORC_WEAK_FURNACE) {
        G = orc_ggx_G1(alpha, cos_o);
    } else {
        if (ci <= 0.0) return 0.0;
        /* wi.m = wo.m > 0 and both cosines with n positive */
        G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, cos_o);
    }
    double one_minus = 1.0 - om;
    *F1 = one_minus * one_minus * one_minus * one_minus * one_minus;
    return G * om / (cos_o * cm);
}

/*
 * Bake the shading terms of the points listed in idx (global indices into
 * the point planes).  Output planes per listed point, [3 + 6K][n_idx]:
 *   Ld(3), Ls0 for k = 0..K-1 (3 each), Ls1 for k = 0..K-1 (3 each).
 * lo/hi: the envelope over single-precision-ambiguous ray outcomes.
 * sq: sum over samples of the squared per-sample contribution divided by
 * spp^2 (so sq - mean^2/spp estimates the variance of the mean).
 */
int orc_bake(void* sp, const float* pts, const int32_t* ptri, int64_t stride,
             const int64_t* idx, int64_t n_idx, int spp_d, int spp_s, int K,
             const double* sigma, uint64_t seed, double eps, int flags,
             int n_threads, double* out, double* lo, double* hi, double* sq,
             int64_t* n_ambiguous)
{
    const scene_t* S = (const scene_t*)sp;
    const int P = 3 + 6 * K;
    int64_t total_ambig = 0;
    int overflow = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel reduction(+ : total_ambig) reduction(| : overflow)
    {
        cast_t* h = (cast_t*)malloc(sizeof(cast_t));
        double acc[3 + 6 * 16], alo[3 + 6 * 16], ahi[3 + 6 * 16], asq[3 + 6 * 16];
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n_idx; ++q) {
            int64_t p = idx[q];
            for (int k = 0; k < P; ++k) acc[k] = alo[k] = ahi[k] = asq[k] = 0.0;
            double x[3], n[3], wo[3];
            for (int k = 0; k < 3; ++k) {
                x[k] = (double)pts[k * stride + p];
                n[k] = (double)pts[(3 + k) * stride + p];
                wo[k] = (double)pts[(6 + k) * stride + p];
            }
            double cos_o = dot3(n, wo);
            if (ptri[p] >= 0 && cos_o < 0.0) {
                for (int k = 0; k < 3; ++k) n[k] = -n[k];
                cos_o = -cos_o;
            }
            if (ptri[p] >= 0 && cos_o > 0.0) {
                double t[3], b[3], o[3];
                orc_frame(n, t, b);
                for (int k = 0; k < 3; ++k) o[k] = x[k] + eps * n[k];
                /* diffuse lobe: cosine-weighted directions, weight 1 */
                for (int s = 0; s < spp_d; ++s) {
                    double xi1, xi2, l[3], wi[3], R[3], Rl[3], Rh[3];
                    sample_uniforms(seed, p, 0, s, spp_d, &xi1, &xi2);
                    orc_sample_cosine(xi1, xi2, l);
                    to_world(t, b, n, l, wi);
                    if (flags & ORC_WEAK_FURNACE) {
                        R[0] = R[1] = R[2] = Rl[0] = Rl[1] = Rl[2] = Rh[0] = Rh[1] = Rh[2] = 1.0;
                    } else {
                        cast(S, o, wi, h);
                        overflow |= h->overflow;
                        total_ambig += radiance_envelope(S, h, R, Rl, Rh);
                    }
                    for (int c = 0; c < 3; ++c) {
                        acc[c] += R[c];
                        alo[c] += Rl[c];
                        ahi[c] += Rh[c];
                        asq[c] += R[c] * R[c];
                    }
                }
                /* specular lobes, one per roughness level */
                for (int k = 0; k < K; ++k) {
                    double alpha = sigma[k] * sigma[k];
                    for (int s = 0; s < spp_s; ++s) {
                        double xi1, xi2, l[3], m[3], wi[3], F1 = 0.0;
                        sample_uniforms(seed, p, 1 + k, s, spp_s, &xi1, &xi2);
                        orc_sample_ggx(alpha, xi1, xi2, l);
                        to_world(t, b, n, l, m);
                        double w = spec_weight(alpha, n, wo, cos_o, m, wi, &F1, flags);
                        if (w == 0.0) continue;
                        double R[3], Rl[3], Rh[3];
                        if (flags & ORC_WEAK_FURNACE) {
                            R[0] = R[1] = R[2] = Rl[0] = Rl[1] = Rl[2] = Rh[0] = Rh[1] = Rh[2] = 1.0;
                        } else {
                            cast(S, o, wi, h);
                            overflow |= h->overflow;
                            total_ambig += radiance_envelope(S, h, R, Rl, Rh);
                        }
                        double F0 = 1.0 - F1;
                        int j0 = 3 + 3 * k, j1 = 3 + 3 * K + 3 * k;
                        for (int c = 0; c < 3; ++c) {
                            acc[j0 + c] += R[c] * F0 * w;
                            alo[j0 + c] += Rl[c] * F0 * w;
                            ahi[j0 + c] += Rh[c] * F0 * w;
                            asq[j0 + c] += (R[c] * F0 * w) * (R[c] * F0 * w);
                            acc[j1 + c] += R[c] * F1 * w;
                            alo[j1 + c] += Rl[c] * F1 * w;
                            ahi[j1 + c] += Rh[c] * F1 * w;
                            asq[j1 + c] += (R[c] * F1 * w) * (R[c] * F1 * w);
                        }
                    }
                }
            }
            for (int k = 0; k < P; ++k) {
                double cnt = (k < 3) ? (double)spp_d : (double)spp_s;
                out[k * n_idx + q] = acc[k] / cnt;
                if (lo) lo[k * n_idx + q] = alo[k] / cnt;
                if (hi) hi[k * n_idx + q] = ahi[k] / cnt;
                if (sq) sq[k * n_idx + q] = asq[k] / (cnt * cnt);
            }
        }
        free(h);
    }
    if (n_ambiguous) *n_ambiguous = total_ambig;
    return overflow ? ORC_EOVERFLOW : 0;
}

/* ---------------------------------------------------------------------- */
/* deterministic quadrature of one shading integral at one point           */
/* ---------------------------------------------------------------------- */
/*
 * lobe < 0: Ld = integral of Li (n.wi)/pi over the hemisphere, midpoint rule
 *           in (theta, phi) with d(omega) = sin(theta) d(theta) d(phi).
 * lobe >= 0: alpha = sigma^2; Ls0 and Ls1 integrated over half vectors m,
 *           using d(omega_i) = 4 (wo.m) d(omega_m), so the integrand
 *           Li F{0,1} D G / (4 n.wo) d(omega_i) becomes
 *           Li F{0,1} D G (wo.m) / (n.wo) d(omega_m); theta_m is stretched
 *           as theta_m = (pi/2) s^4 so narrow lobes are resolved.
 * out: [6] = Ld rgb (lobe < 0) or Ls0 rgb, Ls1 rgb.
 */
int orc_quadrature(void* sp, const double* x, const double* nrm, const double* wo,
                   int lobe, double sigma, int n_theta, int n_phi, double eps,
                   double* out)
{
    const scene_t* S = (const scene_t*)sp;
    cast_t* h = (cast_t*)malloc(sizeof(cast_t));
    double n[3] = {nrm[0], nrm[1], nrm[2]}, t[3], b[3], o[3];
    double cos_o = dot3(n, wo);
    orc_frame(n, t, b);
    for (int k = 0; k < 3; ++k) o[k] = x[k] + eps * n[k];
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    int overflow = 0;
    double dphi = 2.0 * ORC_PI / n_phi;
    if (lobe < 0) {
        double dth = 0.5 * ORC_PI / n_theta;
        for (int i = 0; i < n_theta; ++i) {
            double th = (i + 0.5) * dth;
            for (int j = 0; j < n_phi; ++j) {
                double ph = (j + 0.5) * dphi;
                double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)}, wi[3], R[3];
                to_world(t, b, n, l, wi);
                cast(S, o, wi, h);
                overflow |= h->overflow;
                radiance(S, &h->nominal, 0, R);
                double wgt = cos(th) / ORC_PI * sin(th) * dth * dphi;
                for (int c = 0; c < 3; ++c) out[c] += R[c] * wgt;
            }
        }
    } else {
        double alpha = sigma * sigma;
        double ds = 1.0 / n_theta;
        for (int i = 0; i < n_theta; ++i) {
            double s = (i + 0.5) * ds;
            double th = 0.5 * ORC_PI * s * s * s * s;
            double dth = 0.5 * ORC_PI * 4.0 * s * s * s * ds;
            double cm = cos(th), D = orc_ggx_D(alpha, cm);
            for (int j = 0; j < n_phi; ++j) {
                double ph = (j + 0.5) * dphi;
                double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cm}, m[3], wi[3];
                to_world(t, b, n, l, m);
                double om = dot3(wo, m);
                if (om <= 0.0) continue;
                for (int k = 0; k < 3; ++k) wi[k] = 2.0 * om * m[k] - wo[k];
                double ci = dot3(n, wi);
                if (ci <= 0.0) continue;
                double G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, cos_o);
                double F1 = pow(1.0 - om, 5.0), F0 = 1.0 - F1;
                double R[3];
                cast(S, o, wi, h);
                overflow |= h->overflow;
                radiance(S, &h->nominal, 0, R);
                double wgt = D * G * om / cos_o * sin(th) * dth * dphi;
                for (int c = 0; c < 3; ++c) {
                    out[c] += R[c] * F0 * wgt;
                    out[3 + c] += R[c] * F1 * wgt;
                }
            }
        }
    }
    free(h);
    return overflow ? ORC_EOVERFLOW : 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* stage-3 path-traced shading refinement (Sec. 4.3, Eq. 10 and 11)       */
/* ---------------------------------------------------------------------- */
/*
 * The shading integrals are re-estimated by growing each stage-1 path
 * (Eq. 9 is its one-vertex case) through glossy surfaces: the first
 * direction and its weight come from the lobe g of the shading exactly as
 * in the bake; at each hit x_i
 *   - an emitter (a triangle with some channel of Le > 0) returns Le and
 *     ends the path (an emitter reflects nothing);
 *   - otherwise the current material (a, sigma, m) at x_i is read from a
 *     trilinear grid; sigma > sigma_diffuse (0.6), or the last allowed
 *     vertex, returns the radiance cache L'(x_i) and ends the path;
 *   - otherwise the path continues with the full BRDF f of Eq. 1 at x_i
 *     (cosine included): the radiance arriving at x_i is estimated by
 *     multiple importance sampling of two strategies, a point drawn on an
 *     emitter (uniform over emitter triangles, uniform on the triangle) and
 *     a direction drawn from f (GGX half vectors or cosine-weighted, one
 *     half each), combined by the balance heuristic; the BRDF direction is
 *     also the one the path continues along.
 * A flag turns emitter sampling off (BRDF sampling only, weight one).
 *
 * At a glossy vertex local directions are taken in the frame (t, b, n) with
 * t the unit first edge of the hit triangle and b = n x t.
 * Random numbers: the first direction uses the stage-1 uniforms of
 * (p, lobe, s); vertex i >= 1 draws two Philox blocks with counter
 * (p lo, p hi, lobe | i << 8 | k << 16, s), k = 0 for the emitter choice
 * (word 0, as floor(u0 n_emit / 2^32)), the point on it (words 1, 2) and
 * the lobe choice (word 3), k = 1 for the direction (words 0, 1); a
 * uniform is (u >> 8) 2^-24.
 *
 * Envelope: every ray cast and every sigma threshold decision along a path
 * is an event; a cast with more than one possible outcome in single
 * precision, or a sigma within 1e-4 of the threshold, is ambiguous.  The
 * path is re-evaluated with each alternative outcome of each ambiguous
 * event (one at a time, the rest nominal), and [lo, hi] spans them.
 */
#define ORC_REFINE_BSDF_ONLY 1
#define ORC_MAX_EVENTS 64
#define ORC_EINVAL (-1)

typedef struct {
    const float* grid;      /* [5][R^3] a_r a_g a_b sigma m, x fastest */
    int res;
    double lo[3], hi[3];
    double sigma_diffuse;
    int max_vertices;
    int flags;
    int n_emit;             /* emitter triangles, ascending index */
    int32_t* emit;
} refine_t;

typedef struct {
    int flip_event;         /* event whose outcome is replaced, -1: none */
    int flip_choice;        /* candidate index (a cast); a decision is inverted */
    int n_events;
    int alts[ORC_MAX_EVENTS];   /* alternatives of each event of the run */
    int overflow;
} pathrun_t;

static double unif24(uint32_t u) { return (double)(u >> 8) / 16777216.0; }

static void vertex_philox(uint64_t seed, int64_t p, int lobe, int s, int vertex, int k,
                          uint32_t u[4])
{
    uint32_t c[4] = {(uint32_t)(uint64_t)p, (uint32_t)((uint64_t)p >> 32),
                     (uint32_t)lobe | ((uint32_t)vertex << 8) | ((uint32_t)k << 16), (uint32_t)s};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    philox(c, key, u);
}

/* Material at x: trilinear interpolation of the grid, nodes at
 * lo + i (hi - lo) / (R - 1), coordinates clamped onto the box. */
static void material_at(const refine_t* M, const double x[3], double mat[5])
{
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double u = (x[a] - M->lo[a]) / (M->hi[a] - M->lo[a]) * (M->res - 1);
        u = fmin(fmax(u, 0.0), (double)(M->res - 1));
        int i = (int)floor(u);
        if (i > M->res - 2) i = M->res - 2;
        i0[a] = i;
        f[a] = u - i;
    }
    int64_t R = M->res, plane = R * R * R;
    for (int c = 0; c < 5; ++c) {
        double v = 0.0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double w = (dx ? f[0] : 1 - f[0]) * (dy ? f[1] : 1 - f[1]) * (dz ? f[2] : 1 - f[2]);
                    int64_t node = (i0[0] + dx) + R * ((i0[1] + dy) + R * (int64_t)(i0[2] + dz));
                    v += w * (double)M->grid[c * plane + node];
                }
        mat[c] = v;
    }
}

static int is_emitter(const scene_t* S, int64_t f)
{
    return S->emission[f] > 0.0 || S->emission[S->T + f] > 0.0 || S->emission[2 * S->T + f] > 0.0;
}

/* The BRDF of Eq. 1 with the cosine: kd/pi (n.wi) + F D G / (4 n.wo),
 * F = ks F0 + F1 (Schlick split of Eq. 7), for unit n, wi, wo; zero unless
 * both directions are above the surface. */
static void brdf_f(const double n[3], const double wo[3], const double wi[3], const double a[3],
                   double alpha, double m, double out[3])
{
    double ci = dot3(n, wi), co = dot3(n, wo);
    out[0] = out[1] = out[2] = 0.0;
    if (ci <= 0.0 || co <= 0.0) return;
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    double hl = norm3(h);
    for (int k = 0; k < 3; ++k) h[k] /= hl;
    double nh = dot3(n, h), hi = dot3(h, wi);
    double spec_base = 0.0, F1 = 0.0;
    if (nh > 0.0 && hi > 0.0) {
        double G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, co);
        spec_base = orc_ggx_D(alpha, nh) * G / (4.0 * co);
        double om = 1.0 - hi;
        F1 = om * om * om * om * om;
    }
    for (int c = 0; c < 3; ++c) {
        double kd = a[c] * (1.0 - m), ks = 0.04 * (1.0 - m) + a[c] * m;
        out[c] = kd / ORC_PI * ci + (ks * (1.0 - F1) + F1) * spec_base;
    }
}

/* Density of the BRDF sampling at a glossy vertex: one half GGX half
 * vectors (D(h)(n.h) / (4 wo.h) in wi), one half cosine-weighted. */
static double brdf_pdf(const double n[3], const double wo[3], const double wi[3], double alpha)
{
    double ci = dot3(n, wi);
    if (ci <= 0.0) return 0.0;
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    double hl = norm3(h);
    for (int k = 0; k < 3; ++k) h[k] /= hl;
    double nh = dot3(n, h), oh = dot3(wo, h);
    double ps = (nh > 0.0 && oh > 0.0) ? orc_ggx_D(alpha, nh) * nh / (4.0 * oh) : 0.0;
    return 0.5 * ps + 0.5 * ci / ORC_PI;
}

/* Unit face normal of triangle f and its area. */
static double face_normal(const scene_t* S, int64_t f, double n[3])
{
    cross3(S->e1 + 3 * f, S->e2 + 3 * f, n);
    double l = norm3(n);
    for (int k = 0; k < 3; ++k) n[k] /= l;
    return 0.5 * l;
}

/* One cast as an event of the run: the nominal outcome, or the chosen
 * alternative when this event is the one being flipped. */
static hit_t path_cast(const scene_t* S, const double o[3], const double d[3], pathrun_t* run,
                       cast_t* h, int* clamp)
{
    cast(S, o, d, h);
    run->overflow |= h->overflow;
    int e = run->n_events++;
    int amb = h->n_cand > 1 || (h->n_cand == 1 && h->cand[0].tri != h->nominal.tri);
    if (e < ORC_MAX_EVENTS) run->alts[e] = amb ? h->n_cand : 0;
    else run->overflow = 1;
    if (e == run->flip_event) {
        *clamp = 1;
        return h->cand[run->flip_choice];
    }
    *clamp = 0;
    return h->nominal;
}

/* Radiance arriving at the start of the ray (o, d) along a refined path
 * (Eq. 10 and 11), the factor of the first lobe weight excluded. */
static void refine_path(const scene_t* S, const refine_t* M, uint64_t seed, int64_t p, int lobe,
                        int s, const double o0[3], const double d0[3], double eps, pathrun_t* run,
                        cast_t* h, double C[3])
{
    double o[3] = {o0[0], o0[1], o0[2]}, d[3] = {d0[0], d0[1], d0[2]};
    double T[3] = {1.0, 1.0, 1.0};
    double pb_prev = -1.0;   /* density of the BRDF sampling that chose d; < 0: the lobe g */
    int nee = !(M->flags & ORC_REFINE_BSDF_ONLY) && M->n_emit > 0;
    C[0] = C[1] = C[2] = 0.0;
    for (int vert = 1;; ++vert) {
        int clamp;
        hit_t hit = path_cast(S, o, d, run, h, &clamp);
        if (hit.tri < 0) return;
        int64_t f = hit.tri;
        if (is_emitter(S, f)) {
            double w = 1.0;
            if (pb_prev >= 0.0 && nee) {
                double nz[3];
                double area = face_normal(S, f, nz);
                double cz = fabs(dot3(nz, d));
                double pl = cz > 0.0 ? hit.t * hit.t / (cz * M->n_emit * area) : INFINITY;
                w = pb_prev / (pb_prev + pl);
            }
            for (int c = 0; c < 3; ++c) C[c] += T[c] * S->emission[c * S->T + f] * w;
            return;
        }
        double y[3], ny[3], wo[3], mat[5];
        for (int k = 0; k < 3; ++k) {
            y[k] = o[k] + hit.t * d[k];
            wo[k] = -d[k];
        }
        face_normal(S, f, ny);
        if (dot3(ny, wo) < 0.0)
            for (int k = 0; k < 3; ++k) ny[k] = -ny[k];
        if (!(dot3(ny, wo) > 0.0)) return;
        material_at(M, y, mat);
        int diffuse = mat[3] > M->sigma_diffuse;
        int e = run->n_events++;
        if (e < ORC_MAX_EVENTS) run->alts[e] = fabs(mat[3] - M->sigma_diffuse) <= 1e-4 ? 1 : 0;
        else run->overflow = 1;
        if (e == run->flip_event) diffuse = !diffuse;
        if (diffuse || vert >= M->max_vertices) {
            double R[3];
            radiance(S, &hit, clamp, R);
            for (int c = 0; c < 3; ++c) C[c] += T[c] * R[c];
            return;
        }
        /* a glossy vertex: BRDF of the current material */
        double sg = fmin(fmax(mat[3], 0.02), 1.0), alpha = sg * sg;
        double a[3] = {mat[0], mat[1], mat[2]}, met = mat[4];
        double yo[3];
        for (int k = 0; k < 3; ++k) yo[k] = y[k] + eps * ny[k];
        uint32_t u[4], v[4];
        vertex_philox(seed, p, lobe, s, vert, 0, u);
        vertex_philox(seed, p, lobe, s, vert, 1, v);
        if (nee) {
            int k_e = (int)(((uint64_t)u[0] * (uint64_t)M->n_emit) >> 32);
            int64_t fe = M->emit[k_e];
            double su = sqrt(unif24(u[1])), b1 = su * (1.0 - unif24(u[2])), b2 = su * unif24(u[2]);
            double z[3], l[3];
            for (int k = 0; k < 3; ++k)
                z[k] = S->v0[3 * fe + k] + b1 * S->e1[3 * fe + k] + b2 * S->e2[3 * fe + k];
            for (int k = 0; k < 3; ++k) l[k] = z[k] - yo[k];
            double dist = norm3(l);
            for (int k = 0; k < 3; ++k) l[k] /= dist;
            double nz[3];
            double area = face_normal(S, fe, nz);
            double cz = fabs(dot3(nz, l));
            if (dot3(ny, l) > 0.0 && cz > 0.0) {
                int cl2;
                hit_t sh = path_cast(S, yo, l, run, h, &cl2);
                if (sh.tri == fe) {
                    double fv[3];
                    brdf_f(ny, wo, l, a, alpha, met, fv);
                    double pl = dist * dist / (cz * M->n_emit * area);
                    double pb = brdf_pdf(ny, wo, l, alpha);
                    for (int c = 0; c < 3; ++c)
                        C[c] += T[c] * fv[c] * S->emission[c * S->T + fe] / (pl + pb);
                }
            }
        }
        /* the path goes on along a direction drawn from f, in the frame of
         * the hit triangle's first edge: t = e1 / |e1|, b = n x t (no sign
         * decision on n, whose components a single-precision cross product
         * of the edges may leave a hair from zero) */
        double t_[3], b_[3], loc[3], w2[3];
        double el = norm3(S->e1 + 3 * f);
        for (int k = 0; k < 3; ++k) t_[k] = S->e1[3 * f + k] / el;
        cross3(ny, t_, b_);
        if (unif24(u[3]) < 0.5) {
            double mh[3];
            orc_sample_ggx(alpha, unif24(v[0]), unif24(v[1]), loc);
            to_world(t_, b_, ny, loc, mh);
            double om = dot3(wo, mh);
            if (om <= 0.0) return;
            for (int k = 0; k < 3; ++k) w2[k] = 2.0 * om * mh[k] - wo[k];
        } else {
            orc_sample_cosine(unif24(v[0]), unif24(v[1]), loc);
            to_world(t_, b_, ny, loc, w2);
        }
        if (dot3(ny, w2) <= 0.0) return;
        double pb = brdf_pdf(ny, wo, w2, alpha);
        if (!(pb > 0.0)) return;
        double fv[3];
        brdf_f(ny, wo, w2, a, alpha, met, fv);
        for (int c = 0; c < 3; ++c) T[c] *= fv[c] / pb;
        for (int k = 0; k < 3; ++k) {
            o[k] = yo[k];
            d[k] = w2[k];
        }
        pb_prev = pb;
    }
}

/* One sample's contribution with its envelope over single flips of
 * ambiguous events.  Returns 1 if some event was ambiguous. */
static int refine_sample(const scene_t* S, const refine_t* M, uint64_t seed, int64_t p, int lobe,
                         int s, const double o[3], const double d[3], double eps, cast_t* h,
                         double C[3], double Cl[3], double Ch[3], int* overflow)
{
    pathrun_t run;
    memset(&run, 0, sizeof(run));
    run.flip_event = -1;
    refine_path(S, M, seed, p, lobe, s, o, d, eps, &run, h, C);
    *overflow |= run.overflow;
    for (int c = 0; c < 3; ++c) Cl[c] = Ch[c] = C[c];
    int n_ev = run.n_events < ORC_MAX_EVENTS ? run.n_events : ORC_MAX_EVENTS;
    int alts[ORC_MAX_EVENTS];
    memcpy(alts, run.alts, sizeof(int) * n_ev);
    int amb = 0;
    for (int e = 0; e < n_ev; ++e) {
        for (int k = 0; k < alts[e]; ++k) {
            pathrun_t r2;
            memset(&r2, 0, sizeof(r2));
            r2.flip_event = e;
            r2.flip_choice = k;
            double A[3];
            refine_path(S, M, seed, p, lobe, s, o, d, eps, &r2, h, A);
            *overflow |= r2.overflow;
            for (int c = 0; c < 3; ++c) {
                Cl[c] = fmin(Cl[c], A[c]);
                Ch[c] = fmax(Ch[c], A[c]);
            }
            amb = 1;
        }
    }
    return amb;
}

/*
 * Refined shading terms of the listed points, laid out as orc_bake's.
 * grid: [5][res^3] material (a_r, a_g, a_b, sigma, m) over [glo, ghi].
 * Returns 0, ORC_EOVERFLOW, or ORC_EINVAL (voxel cache, which the
 * refinement does not take, or bad arguments).
 */
int orc_refine(void* sp, const float* pts, const int32_t* ptri, int64_t stride, const int64_t* idx,
               int64_t n_idx, int spp_d, int spp_s, int K, const double* sigma, uint64_t seed,
               double eps, const float* grid, int res, const double* glo, const double* ghi,
               double sigma_diffuse, int max_vertices, int flags, int n_threads, double* out,
               double* lo, double* hi, double* sq, int64_t* n_ambiguous)
{
    const scene_t* S = (const scene_t*)sp;
    if (S->cache_kind == 2 || res < 2 || max_vertices < 1 || max_vertices > 16) return ORC_EINVAL;
    refine_t M;
    memset(&M, 0, sizeof(M));
    M.grid = grid;
    M.res = res;
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = glo[a];
        M.hi[a] = ghi[a];
    }
    M.sigma_diffuse = sigma_diffuse;
    M.max_vertices = max_vertices;
    M.flags = flags;
    M.emit = (int32_t*)malloc(sizeof(int32_t) * (S->T > 0 ? S->T : 1));
    for (int64_t f = 0; f < S->T; ++f)
        if (is_emitter(S, f)) M.emit[M.n_emit++] = (int32_t)f;
    const int P = 3 + 6 * K;
    int64_t total_ambig = 0;
    int overflow = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel reduction(+ : total_ambig) reduction(| : overflow)
    {
        cast_t* h = (cast_t*)malloc(sizeof(cast_t));
        double acc[3 + 6 * 16], alo[3 + 6 * 16], ahi[3 + 6 * 16], asq[3 + 6 * 16];
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n_idx; ++q) {
            int64_t p = idx[q];
            for (int k = 0; k < P; ++k) acc[k] = alo[k] = ahi[k] = asq[k] = 0.0;
            double x[3], n[3], wo[3];
            for (int k = 0; k < 3; ++k) {
                x[k] = (double)pts[k * stride + p];
                n[k] = (double)pts[(3 + k) * stride + p];
                wo[k] = (double)pts[(6 + k) * stride + p];
            }
            double cos_o = dot3(n, wo);
            if (ptri[p] >= 0 && cos_o < 0.0) {
                for (int k = 0; k < 3; ++k) n[k] = -n[k];
                cos_o = -cos_o;
            }
            if (ptri[p] >= 0 && cos_o > 0.0) {
                double t[3], b[3], o[3];
                orc_frame(n, t, b);
                for (int k = 0; k < 3; ++k) o[k] = x[k] + eps * n[k];
                for (int s = 0; s < spp_d; ++s) {
                    double xi1, xi2, l[3], wi[3], R[3], Rl[3], Rh[3];
                    sample_uniforms(seed, p, 0, s, spp_d, &xi1, &xi2);
                    orc_sample_cosine(xi1, xi2, l);
                    to_world(t, b, n, l, wi);
                    total_ambig += refine_sample(S, &M, seed, p, 0, s, o, wi, eps, h, R, Rl, Rh,
                                                 &overflow);
                    for (int c = 0; c < 3; ++c) {
                        acc[c] += R[c];
                        alo[c] += Rl[c];
                        ahi[c] += Rh[c];
                        asq[c] += R[c] * R[c];
                    }
                }
                for (int k = 0; k < K; ++k) {
                    double alpha = sigma[k] * sigma[k];
                    for (int s = 0; s < spp_s; ++s) {
                        double xi1, xi2, l[3], m[3], wi[3], F1 = 0.0;
                        sample_uniforms(seed, p, 1 + k, s, spp_s, &xi1, &xi2);
                        orc_sample_ggx(alpha, xi1, xi2, l);
                        to_world(t, b, n, l, m);
                        double w = spec_weight(alpha, n, wo, cos_o, m, wi, &F1, 0);
                        if (w == 0.0) continue;
                        double R[3], Rl[3], Rh[3];
                        total_ambig += refine_sample(S, &M, seed, p, 1 + k, s, o, wi, eps, h, R, Rl,
                                                     Rh, &overflow);
                        double F0 = 1.0 - F1;
                        int j0 = 3 + 3 * k, j1 = 3 + 3 * K + 3 * k;
                        for (int c = 0; c < 3; ++c) {
                            acc[j0 + c] += R[c] * F0 * w;
                            alo[j0 + c] += Rl[c] * F0 * w;
                            ahi[j0 + c] += Rh[c] * F0 * w;
                            asq[j0 + c] += (R[c] * F0 * w) * (R[c] * F0 * w);
                            acc[j1 + c] += R[c] * F1 * w;
                            alo[j1 + c] += Rl[c] * F1 * w;
                            ahi[j1 + c] += Rh[c] * F1 * w;
                            asq[j1 + c] += (R[c] * F1 * w) * (R[c] * F1 * w);
                        }
                    }
                }
            }
            for (int k = 0; k < P; ++k) {
                double cnt = (k < 3) ? (double)spp_d : (double)spp_s;
                out[k * n_idx + q] = acc[k] / cnt;
                if (lo) lo[k * n_idx + q] = alo[k] / cnt;
                if (hi) hi[k * n_idx + q] = ahi[k] / cnt;
                if (sq) sq[k * n_idx + q] = asq[k] / (cnt * cnt);
            }
        }
        free(h);
    }
    free(M.emit);
    if (n_ambiguous) *n_ambiguous = total_ambig;
    return overflow ? ORC_EOVERFLOW : 0;
}

/* Test hooks: the BRDF, its sampling density and the material lookup. */
void orc_brdf(const double* n, const double* wo, const double* wi, const double* a, double sigma,
              double m, double* out)
{
    double sg = fmin(fmax(sigma, 0.02), 1.0);
    brdf_f(n, wo, wi, a, sg * sg, m, out);
}

double orc_brdf_pdf(const double* n, const double* wo, const double* wi, double sigma)
{
    double sg = fmin(fmax(sigma, 0.02), 1.0);
    return brdf_pdf(n, wo, wi, sg * sg);
}

/* Radiance a path ends on at hit `hit` seen along d, for the quadrature
 * below: Le at an emitter, L' at a diffuse hit (sigma > sigma_diffuse),
 * and -1 in out[3] at a glossy hit (the caller integrates further). */
static void end_radiance(const scene_t* S, const refine_t* M, const hit_t* hit, const double o[3],
                         const double d[3], double out[4], double mat[5])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (hit->tri < 0) return;
    if (is_emitter(S, hit->tri)) {
        for (int c = 0; c < 3; ++c) out[c] = S->emission[c * S->T + hit->tri];
        return;
    }
    double y[3];
    for (int k = 0; k < 3; ++k) y[k] = o[k] + hit->t * d[k];
    material_at(M, y, mat);
    if (mat[3] > M->sigma_diffuse) {
        radiance(S, hit, 0, out);
        out[3] = 0.0;
        return;
    }
    out[3] = -1.0;
}

/* The radiance leaving a glossy hit y (normal ny facing wo, material mat)
 * toward wo, as the integral of f times the radiance its directions end on
 * (Eq. 10 with paths of one more vertex): the diffuse part of f by a
 * midpoint rule in (theta, phi) about ny, the specular part over half
 * vectors (d omega_i = 4 (wo.m) d omega_m, theta_m = (pi/2) s^4).  The
 * weight of directions that reach a further glossy surface is added to
 * *deeper. */
static void glossy_integral(const scene_t* S, const refine_t* M, cast_t* h, const double y[3],
                            const double ny[3], const double wo[3], const double mat[5], double eps,
                            int nt, int np, double L[3], double* deeper)
{
    double t[3], b[3], yo[3];
    orc_frame(ny, t, b);
    for (int k = 0; k < 3; ++k) yo[k] = y[k] + eps * ny[k];
    double sg = fmin(fmax(mat[3], 0.02), 1.0), alpha = sg * sg, met = mat[4];
    double co = dot3(ny, wo);
    L[0] = L[1] = L[2] = 0.0;
    double dphi = 2.0 * ORC_PI / np;
    /* diffuse part: kd / pi (n.wi) */
    double dth = 0.5 * ORC_PI / nt;
    for (int i = 0; i < nt; ++i) {
        double th = (i + 0.5) * dth;
        for (int j = 0; j < np; ++j) {
            double ph = (j + 0.5) * dphi;
            double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)}, wi[3], R[4], m2[5];
            to_world(t, b, ny, l, wi);
            cast(S, yo, wi, h);
            end_radiance(S, M, &h->nominal, yo, wi, R, m2);
            double wgt = cos(th) / ORC_PI * sin(th) * dth * dphi;
            if (R[3] < 0.0) {
                *deeper += wgt;
                continue;
            }
            for (int c = 0; c < 3; ++c) L[c] += mat[c] * (1.0 - met) * R[c] * wgt;
        }
    }
    /* specular part: (ks F0 + F1) D G / (4 n.wo) */
    double ds = 1.0 / nt;
    for (int i = 0; i < nt; ++i) {
        double s = (i + 0.5) * ds;
        double th = 0.5 * ORC_PI * s * s * s * s;
        double dthm = 0.5 * ORC_PI * 4.0 * s * s * s * ds;
        double cm = cos(th), D = orc_ggx_D(alpha, cm);
        for (int j = 0; j < np; ++j) {
            double ph = (j + 0.5) * dphi;
            double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cm}, m[3], wi[3];
            to_world(t, b, ny, l, m);
            double om = dot3(wo, m);
            if (om <= 0.0) continue;
            for (int k = 0; k < 3; ++k) wi[k] = 2.0 * om * m[k] - wo[k];
            double ci = dot3(ny, wi);
            if (ci <= 0.0) continue;
            double G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, co);
            double F1 = pow(1.0 - om, 5.0);
            double R[4], m2[5];
            cast(S, yo, wi, h);
            end_radiance(S, M, &h->nominal, yo, wi, R, m2);
            double wgt = D * G * om / co * sin(th) * dthm * dphi;
            if (R[3] < 0.0) {
                *deeper += wgt;
                continue;
            }
            for (int c = 0; c < 3; ++c) {
                double ks = 0.04 * (1.0 - met) + mat[c] * met;
                L[c] += (ks * (1.0 - F1) + F1) * R[c] * wgt;
            }
        }
    }
}

/*
 * Deterministic quadrature of one refined shading integral at one point
 * (the expectation the Monte Carlo refinement estimates), for scenes in
 * which every path ends by its second vertex: the outer integral over the
 * lobe g as orc_quadrature takes it (lobe < 0: Ld; lobe >= 0: Ls0, Ls1 at
 * roughness sigma), the radiance of a glossy first hit by glossy_integral.
 * out[6]: the three or six values; out[6]: the weight of directions that
 * went deeper than two vertices (zero when the scene is as required).
 */
int orc_refine_quadrature(void* sp, const double* x, const double* nrm, const double* wo, int lobe,
                          double sigma, const float* grid, int res, const double* glo,
                          const double* ghi, double sigma_diffuse, int n_theta, int n_phi,
                          int n_theta2, int n_phi2, double eps, double* out)
{
    const scene_t* S = (const scene_t*)sp;
    refine_t M;
    memset(&M, 0, sizeof(M));
    M.grid = grid;
    M.res = res;
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = glo[a];
        M.hi[a] = ghi[a];
    }
    M.sigma_diffuse = sigma_diffuse;
    M.max_vertices = 2;
    double n[3] = {nrm[0], nrm[1], nrm[2]}, t[3], b[3], o[3];
    double cos_o = dot3(n, wo);
    orc_frame(n, t, b);
    for (int k = 0; k < 3; ++k) o[k] = x[k] + eps * n[k];
    double acc[6] = {0, 0, 0, 0, 0, 0}, deeper = 0.0;
    int overflow = 0;
    double dphi = 2.0 * ORC_PI / n_phi;
#pragma omp parallel reduction(+ : deeper) reduction(| : overflow)
    {
        cast_t* h = (cast_t*)malloc(sizeof(cast_t));
        double loc[6] = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n_theta; ++i) {
            for (int j = 0; j < n_phi; ++j) {
                double ph = (j + 0.5) * dphi, th, wgt_d = 0.0, wi[3], F1 = 0.0, wgt_s = 0.0;
                if (lobe < 0) {
                    double dth = 0.5 * ORC_PI / n_theta;
                    th = (i + 0.5) * dth;
                    double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
                    to_world(t, b, n, l, wi);
                    wgt_d = cos(th) / ORC_PI * sin(th) * dth * dphi;
                } else {
                    double alpha = sigma * sigma, ds = 1.0 / n_theta, s = (i + 0.5) * ds;
                    th = 0.5 * ORC_PI * s * s * s * s;
                    double dthm = 0.5 * ORC_PI * 4.0 * s * s * s * ds;
                    double cm = cos(th);
                    double l[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cm}, m[3];
                    to_world(t, b, n, l, m);
                    double om = dot3(wo, m);
                    if (om <= 0.0) continue;
                    for (int k = 0; k < 3; ++k) wi[k] = 2.0 * om * m[k] - wo[k];
                    double ci = dot3(n, wi);
                    if (ci <= 0.0) continue;
                    double G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, cos_o);
                    F1 = pow(1.0 - om, 5.0);
                    wgt_s = orc_ggx_D(alpha, cm) * G * om / cos_o * sin(th) * dthm * dphi;
                }
                double R[4], mat[5];
                cast(S, o, wi, h);
                overflow |= h->overflow;
                end_radiance(S, &M, &h->nominal, o, wi, R, mat);
                if (R[3] < 0.0) {
                    double y[3], ny[3], w1[3];
                    for (int k = 0; k < 3; ++k) {
                        y[k] = o[k] + h->nominal.t * wi[k];
                        w1[k] = -wi[k];
                    }
                    face_normal(S, h->nominal.tri, ny);
                    if (dot3(ny, w1) < 0.0)
                        for (int k = 0; k < 3; ++k) ny[k] = -ny[k];
                    double dl = 0.0;
                    glossy_integral(S, &M, h, y, ny, w1, mat, eps, n_theta2, n_phi2, R, &dl);
                    deeper += dl * (lobe < 0 ? wgt_d : wgt_s);
                }
                if (lobe < 0) {
                    for (int c = 0; c < 3; ++c) loc[c] += R[c] * wgt_d;
                } else {
                    for (int c = 0; c < 3; ++c) {
                        loc[c] += R[c] * (1.0 - F1) * wgt_s;
                        loc[3 + c] += R[c] * F1 * wgt_s;
                    }
                }
            }
        }
#pragma omp critical
        for (int k = 0; k < 6; ++k) acc[k] += loc[k];
        free(h);
    }
    for (int k = 0; k < 6; ++k) out[k] = acc[k];
    out[6] = deeper;
    return overflow ? ORC_EOVERFLOW : 0;
}

/* Test hook: the refinement's material lookup at n points x[n][3]. */
void orc_material_at(const float* grid, int res, const double* lo, const double* hi,
                     const double* x, int64_t n, double* out)
{
    refine_t M;
    memset(&M, 0, sizeof(M));
    M.grid = grid;
    M.res = res;
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = lo[a];
        M.hi[a] = hi[a];
    }
    for (int64_t i = 0; i < n; ++i) material_at(&M, x + 3 * i, out + 5 * i);
}
