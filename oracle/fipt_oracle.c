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
