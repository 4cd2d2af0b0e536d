/*
 * fipt.h -- C ABI of the MI355X (gfx950) hot path of Factorized Inverse Path
 * Tracing (Wu, Zhu et al., "Factorized Inverse Path Tracing for Efficient and
 * Accurate Material-Lighting Estimation", ICCV 2023).
 *
 * The library bakes the factorized shading terms of Eq. 6 (diffuse shading
 * Ld and the two specular shadings Ls0, Ls1 of the Fresnel split, Eq. 7, at
 * each roughness level of the lerp table, Eq. 8) for a set of surface
 * points, with the stage-1 radiance query of Eq. 9 (incident radiance =
 * radiance cache + per-triangle emission at the first hit along each
 * sampled direction), and evaluates the factored re-render of Eq. 5 with the
 * photometric loss of Eq. 2 / Eq. 15 and its gradient with respect to the
 * per-point material (albedo a, roughness sigma, metallic m).
 *
 * Conventions shared by every call:
 *   - Status: every call returns FIPT_OK (0) or a negative FIPT_E* code; the
 *     text of the last error on the calling thread is fipt_last_error().
 *     All arguments are validated before any work is enqueued.
 *   - Memory: pointers documented "device" must point to memory of the
 *     current HIP device (e.g. a torch CUDA tensor's data_ptr()); "host"
 *     pointers are read during the call only.  Device buffers are borrowed:
 *     the caller keeps them alive until the stream work has completed.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *     Every compute call is asynchronous on that stream.
 *   - Layout: per-point data are structure-of-arrays float planes; plane k of
 *     a buffer starts at base + k * stride elements.
 *   - No call allocates device memory except fipt_scene_create,
 *     fipt_scene_set_voxel_radiance, the plan constructors
 *     (fipt_grid_plan_create, fipt_emission_plan_create,
 *     fipt_voxel_plan_create) and fipt_server_create.
 */
#ifndef FIPT_H
#define FIPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FIPT_OK 0
#define FIPT_EINVAL (-1)     /* invalid argument                              */
#define FIPT_ENOMEM (-2)     /* device or host allocation failed              */
#define FIPT_EHIP (-3)       /* a HIP runtime call failed                      */
#define FIPT_EBUSY (-4)      /* object still referenced by work in flight     */
#define FIPT_EAGAIN (-5)     /* not ready yet (serving poll)                  */
#define FIPT_ECANCELED (-6)  /* request cancelled or timed out                */

#define FIPT_MAX_LEVELS 16   /* maximum number of roughness levels K          */
#define FIPT_LOSS_SLOTS 2049 /* doubles in a render-loss result buffer        */

/* Radiance cache kinds (fipt_scene_set_radiance). */
#define FIPT_CACHE_TRIANGLE 0   /* one RGB value per triangle, [3][T]          */
#define FIPT_CACHE_VERTEX 1     /* one RGB value per vertex, [3][V], linear
                                   (barycentric) interpolation over triangles */
#define FIPT_CACHE_VOXEL 2      /* voxel grid, nearest voxel of the hit point
                                   (fipt_scene_set_voxel_radiance)            */

/* Tone maps of the loss (fipt_render_loss). */
#define FIPT_TONEMAP_NONE 0     /* Gamma(x) = x                                */
#define FIPT_TONEMAP_LOG_SRGB 1 /* Gamma(x) = sRGB-OETF(log(1 + max(x, 0)))    */

typedef struct fipt_scene_s* fipt_scene;
typedef struct fipt_grid_plan_s* fipt_grid_plan;
typedef struct fipt_emission_plan_s* fipt_emission_plan;
typedef struct fipt_voxel_plan_s* fipt_voxel_plan;
typedef struct fipt_server_s* fipt_server;
typedef struct fipt_hashgrid_plan_s* fipt_hashgrid_plan;

/* Pinhole camera: rays leave `pos` through pixel centres; `fwd` is the view
 * direction, `up` fixes the roll, `vfov_deg` the vertical field of view;
 * square pixels; pixel (i, j) (j = 0 the top row) of camera c is point
 * offset(c) + j * width + i, offsets accumulating width * height per camera. */
typedef struct fipt_camera {
    float pos[3];
    float fwd[3];
    float up[3];
    float vfov_deg;
    int32_t width;
    int32_t height;
} fipt_camera;

/* Shading points (the (x, wo) pairs of Eq. 2), device SoA:
 *   planes: 9 float planes px py pz nx ny nz ox oy oz -- position x, unit
 *           geometric normal n facing the viewer, unit direction wo toward
 *           the viewer;
 *   tri:    index of the triangle x lies on, or -1 for "no surface" (the
 *           bake writes zeros for such points);
 *   n:      number of points, 1 <= n < 2^31; stride: elements between
 *           planes (>= n). */
typedef struct fipt_points {
    float* planes;
    int32_t* tri;
    int64_t n;
    int64_t stride;
} fipt_points;

/* Baked shading terms, device SoA, 3 + 6K float planes:
 *   plane 0..2                 Ld (r, g, b)
 *   plane 3 + 3k + c           Ls0 at roughness level k, channel c
 *   plane 3 + 3K + 3k + c      Ls1 at roughness level k, channel c */
typedef struct fipt_shading {
    float* planes;
    int64_t stride;
} fipt_shading;

/* Bake parameters (Eq. 6 estimated by importance-sampled Monte Carlo):
 *   spp_d     samples of the cosine lobe per point, 1..65536;
 *   spp_s     samples of each GGX level per point, 1..65536;
 *   n_levels  K, 1..FIPT_MAX_LEVELS; sigma[0..K-1] strictly increasing in
 *             (0, 1]; the GGX width is alpha = sigma^2;
 *   seed      Philox4x32-10 key; sample s of lobe l (0 = diffuse, 1 + k =
 *             level k) of point p uses counter (p lo, p hi, l, s);
 *   ray_eps   offset of ray origins along n, > 0, scene units;
 *   flags     0. */
typedef struct fipt_bake_params {
    int32_t spp_d;
    int32_t spp_s;
    int32_t n_levels;
    float sigma[FIPT_MAX_LEVELS];
    uint64_t seed;
    float ray_eps;
    int32_t flags;
} fipt_bake_params;

/* Scene summary (fipt_scene_info). */
typedef struct fipt_scene_info {
    int64_t n_tris;
    int64_t n_verts;
    int64_t n_nodes;        /* BVH nodes                                     */
    int64_t device_bytes;   /* resident device memory of the scene           */
    int32_t max_depth;      /* deepest BVH node                              */
    int32_t cache_kind;     /* FIPT_CACHE_* last set, -1 if none             */
    float bmin[3];
    float bmax[3];
} fipt_scene_info;

/* Per-launch traversal counters (fipt_bake_traversal_stats).  The two step
 * counts are per wavefront (one per loop iteration of a whole wavefront), so
 * nodes / (64 node_steps) and tris / (64 tri_steps) are the fractions of
 * lanes doing useful work in the node and triangle loops. */
typedef struct fipt_traversal_stats {
    uint64_t rays;          /* rays cast                                     */
    uint64_t nodes;         /* BVH nodes fetched (lane count)                */
    uint64_t tris;          /* triangles tested (lane count)                 */
    uint64_t hits;          /* rays that hit a surface                       */
    uint64_t node_steps;    /* wavefront iterations of the node loop         */
    uint64_t tri_steps;     /* wavefront iterations of the triangle loop     */
    uint64_t chain_levels;  /* levels of a point's origin chain a ray starts
                               below (lane count; each tests the three
                               siblings of the chain's child)               */
} fipt_traversal_stats;

/* ---- library ----------------------------------------------------------- */

/* Text of the last error on the calling thread (empty if none); valid until
 * the next fipt_* call on that thread. */
const char* fipt_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int32_t fipt_version(void);

/* ---- scene (triangle mesh, BVH, radiance cache, emission) -------------- */

/* Copy a triangle mesh (the scene geometry assumed given, Sec. 3), build a
 * bounding-volume hierarchy on the host and upload it to `device`.
 *   verts: host float [n_verts][3]; tris: host int32 [n_tris][3] vertex
 *   indices (each in [0, n_verts)); 1 <= n_tris < 2^28.
 * The scene owns its device memory until fipt_scene_destroy.  The radiance
 * starts at zero (no cache, no emission).  FIPT_EINVAL on bad sizes or
 * indices, and when the tree would exceed what the traversal addresses
 * (2^24 4-wide nodes: tens of millions of triangles) or holds on its
 * stack; FIPT_ENOMEM on allocation failure, FIPT_EHIP on HIP errors. */
int fipt_scene_create(const float* verts, int64_t n_verts, const int32_t* tris,
                      int64_t n_tris, int32_t device, void* stream, fipt_scene* out);

/* Set the radiance the bake returns at a hit: radiance cache L' (Eq. 9) of
 * kind FIPT_CACHE_TRIANGLE ([3][n_tris]) or FIPT_CACHE_VERTEX ([3][n_verts]),
 * plus per-triangle emission Le ([3][n_tris], NULL = zero).  Both device
 * float planes; read on `stream`, not retained.  FIPT_EBUSY while serving
 * requests reference the scene (their launches read the radiance records
 * this call rewrites); the same holds for fipt_scene_set_emission. */
int fipt_scene_set_radiance(fipt_scene s, int32_t cache_kind, const float* cache,
                            int64_t n_cache, const float* emission, void* stream);

/* Set a voxel-grid radiance cache, the form Sec. 4.2 gives L' (average of
 * the observed pixels per voxel, queried at the nearest voxel): a hit at x
 * reads voxel (i, j, k) = floor((x - bmin) res / (bmax - bmin)) per axis,
 * clamped to [0, res - 1], whose value is cache[c][(k res + j) res + i]
 * (device float [3][cache_stride], cache_stride >= res^3, as written by
 * fipt_voxel_pool), and adds the triangle's emission Le ([3][n_tris],
 * NULL = zero).  1 <= res <= 512; bmin_host < bmax_host (host float [3]),
 * finite.  The scene keeps its own sparse copy (a voxel whose three values
 * are all zero is empty: 16 bytes per 64 voxels plus 16 bytes per occupied
 * voxel, kept until the scene is destroyed or a larger grid is set); the
 * bake reads it until fipt_scene_set_radiance selects another cache.  The
 * call waits for the device to finish earlier work and reads the occupied
 * count back, so it is a set-up call, not one to capture.  On an error the
 * scene is left with no cache (emission only).  Serving
 * (fipt_server_submit) rejects scenes with a voxel cache, and this call
 * returns FIPT_EBUSY while serving requests reference the scene. */
int fipt_scene_set_voxel_radiance(fipt_scene s, const float* cache, int64_t cache_stride,
                                  int32_t res, const float* bmin_host, const float* bmax_host,
                                  const float* emission, void* stream);

/* Replace the per-triangle emission only (device [3][n_tris]); the cache set
 * last is kept.  Used between re-bakes when emitters are re-estimated. */
int fipt_scene_set_emission(fipt_scene s, const float* emission, void* stream);

int fipt_scene_info_get(fipt_scene s, fipt_scene_info* out);

/* Host-only diagnostic: build the BVH of a mesh exactly as
 * fipt_scene_create does, without touching any GPU, and verify it: every
 * triangle appears in exactly one leaf, every child box encloses the
 * triangles below it, and no internal node is deeper than the traversal
 * stack allows.  Writes the node count and the deepest internal node.
 * FIPT_EINVAL (with the violated property in the error text) otherwise. */
int fipt_bvh_validate(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                      int64_t* n_nodes, int32_t* max_depth);

/* Release the scene's device memory.  FIPT_EBUSY while a serving request
 * references it. */
int fipt_scene_destroy(fipt_scene s);

/* ---- ray casting (the closest-hit query of Eq. 9) ----------------------- */

/* Closest hit of each of n rays, the query the bake and the point
 * generation run, exposed for callers that trace their own rays and for
 * checking the traversal against other implementations:
 *   rays:     device float planes [6][stride]: origin x, y, z, direction
 *             x, y, z (any non-zero length); hits have t > 0 along o + t d;
 *   hit_tri:  device int32 [n]: original index of the nearest triangle
 *             (exact ties in t go to the lower index), -1 on a miss;
 *   hit_tuv:  device float planes [3][hit_stride] or NULL: t and the
 *             barycentric weights u, v of the triangle's second and third
 *             vertices (0 on a miss).
 * 1 <= n < 2^31, stride >= n, hit_stride >= n.  Asynchronous on `stream`. */
int fipt_cast_rays(fipt_scene s, const float* rays, int64_t n, int64_t stride, int32_t* hit_tri,
                   float* hit_tuv, int64_t hit_stride, void* stream);

/* ---- shading points ---------------------------------------------------- */

/* For every pixel centre of every camera (host array of n_cams, at most 48
 * per call; offset out->planes / out->tri for more), cast the
 * camera ray and write the closest hit as a shading point: position, face
 * normal flipped toward the camera, wo = -direction, triangle index (-1 on a
 * miss).  out->n must equal the total pixel count. */
int fipt_gen_points(fipt_scene s, const fipt_camera* cams, int32_t n_cams,
                    const fipt_points* out, void* stream);

/* ---- the bake (Eq. 6, 7, 9) --------------------------------------------- */

/* Bake Ld, Ls0[k], Ls1[k] for all points:
 *   Ld    = mean over cosine-distributed directions of R,
 *   Ls0_k = mean over GGX(alpha_k) half vectors m of R F0 w,
 *   Ls1_k = mean over the same of R F1 w,
 * where R = cache + emission at the first hit (0 on a miss),
 * w = G(wi, wo) (wo.m) / ((n.wo)(n.m)) with separable Smith G, F1 =
 * (1 - wi.m)^5, F0 = 1 - F1, and samples with wo.m <= 0 or n.wi <= 0 count
 * as zero.  Each lobe's samples are stratified: the uniforms of sample s
 * come from the s-th of spp equal segments of a curve through the unit
 * square (see fipt_lobe_uniforms).  Points with tri < 0 or n.wo = 0 get zeros.  `out` must hold
 * 3 + 6K planes of at least pts->n elements.  Asynchronous on `stream`;
 * allocates nothing: its work counters come from a ring of 16 slots held by
 * the scene, and the call makes `stream` wait until the previous launch
 * that used the same slot has finished, so concurrent calls on any streams
 * are safe. */
int fipt_bake(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
              const fipt_shading* out, void* stream);

/* The two uniforms (xi1, xi2) in [0, 1) that the bake draws for lobe `lobe`
 * (0 diffuse, k >= 1 roughness level k - 1) and samples s = 0 .. n_samples - 1
 * of the points whose counter indices are p0 .. p0 + n_points - 1, with key
 * `seed`, when the lobe has n = n_samples samples.  With u the
 * Philox4x32-10 block of the counter (p low, p high, lobe, s) and
 * W = floor(2^32 / n), the point U = s W + floor(u0 W / 2^32) on the
 * 32-bit line lies in the s-th of n equal segments.  U's top four bits
 * pick a cell of the 4 x 4 grid along a Hilbert curve from cell (0, 0) to
 * cell (3, 0) (first step toward larger xi2); its other 28 bits, read as a
 * Morton code (even bits to xi1, odd bits to xi2), give the next 14 bits of
 * each coordinate, and the top bytes of u1 and u2 their low 8 bits (each
 * uniform a 24-bit integer times 2^-24).
 * out: device float [2][n_points][n_samples] (xi1 block, then xi2 block).
 * For checking the random streams against other implementations;
 * n_points * n_samples must be in [1, 2^31).  Asynchronous on `stream`. */
int fipt_lobe_uniforms(uint64_t seed, int64_t p0, int64_t n_points, int32_t lobe,
                       int32_t n_samples, float* out, void* stream);

/* Same bake, instrumented: also accumulates traversal counters into
 * `stats_dev` (device, 7 uint64 in fipt_traversal_stats order, added to).
 * Slower than fipt_bake; meant for measuring algorithmic bytes per ray. */
int fipt_bake_traversal_stats(fipt_scene s, const fipt_points* pts,
                              const fipt_bake_params* p, const fipt_shading* out,
                              uint64_t* stats_dev, void* stream);

/* ---- stage-3 path-traced shading refinement (Sec. 4.3, Eq. 10 / 11) ---- */

#define FIPT_REFINE_BSDF_ONLY 1   /* no emitter sampling: BRDF sampling only */

/* The current material estimate and the path rules of the refinement:
 *   material      device float [5][res^3] (a_r, a_g, a_b, sigma, m), node
 *                 (i, j, k) at bmin + (i, j, k) (bmax - bmin) / (res - 1),
 *                 x fastest; read trilinearly at each hit, positions clamped
 *                 onto the box (as fipt_grid_gather); 2 <= res <= 1024;
 *   sigma_diffuse a hit with roughness above it ends the path at the cache
 *                 (the paper's 0.6);
 *   max_vertices  the path ends at the cache at this vertex at the latest,
 *                 1..16 (1 gives the stage-1 bake for non-emitters);
 *   flags         0 or FIPT_REFINE_BSDF_ONLY. */
typedef struct fipt_refine_params {
    const float* material;
    int32_t res;
    float bmin[3];
    float bmax[3];
    float sigma_diffuse;
    int32_t max_vertices;
    int32_t flags;
} fipt_refine_params;

/* Refined shading terms (same layout, sampling and counters as fipt_bake):
 * each lobe sample's first direction and weight are the bake's; the path
 * then grows (Eq. 10): a hit on an emitter (some channel of its emission
 * > 0) returns its emission only; otherwise a hit whose roughness exceeds
 * sigma_diffuse, or the max_vertices-th vertex, returns the radiance cache
 * at the hit (Eq. 11); otherwise the hit is glossy and the radiance leaving
 * it toward the previous vertex is estimated with the BRDF of Eq. 1 (with
 * the cosine; GGX alpha = max(sigma, 0.02)^2): a point on an emitter
 * (emitter triangle uniform by index in ascending original index, point
 * uniform in area) and a direction drawn from f (GGX half vector or cosine,
 * one half each) combined by the balance heuristic, the path continuing
 * along the latter (local directions at a vertex in the frame of its
 * triangle's first edge: t = (v1 - v0) / |v1 - v0|, b = n x t, n the face
 * normal facing the incoming ray).  Vertex i >= 1 of sample s of lobe l of point p draws
 * Philox4x32-10 blocks with counter (p lo, p hi, l | i << 8 | k << 16, s),
 * k = 0 (word 0: the emitter, floor(u n_emitters / 2^32); words 1, 2: the
 * point; word 3: GGX when (u >> 8) 2^-24 < 1/2) and k = 1 (words 0, 1: the
 * direction); uniforms are (u >> 8) 2^-24.  The scene's cache must be per
 * triangle or per vertex (FIPT_EINVAL for a voxel cache).  The call lists
 * the scene's emitters in its own memory first, so refinements of one
 * scene run in call order (the call makes `stream` wait for the previous
 * one).  Allocates nothing; asynchronous on `stream`. */
int fipt_refine(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                const fipt_refine_params* r, const fipt_shading* out, void* stream);

/* ---- factored re-render and loss (Eq. 5, 8, 2 / 15) -------------------- */

/* For n points, with material[5][mat_stride] = (a_r, a_g, a_b, sigma, m) and
 * observed radiance Lgt[3][obs_stride] (device float planes):
 *   kd = a (1 - m), ks = 0.04 (1 - m) + a m,
 *   Ls*(sigma) = lerp between the two levels of sigma_host[0..K-1] that
 *                bracket sigma (clamped outside, right-hand segment at an
 *                interior knot), K >= 2, sigma strictly increasing;
 *   Lr = kd Ld + ks Ls0(sigma) + Ls1(sigma);
 *   loss = sum over points and channels of (Gamma(Lr) - Gamma(Lgt))^2.
 * Writes loss (double, summed in a fixed order: bitwise reproducible) to
 * loss_dev[0]; loss_dev must hold FIPT_LOSS_SLOTS doubles (the rest is
 * scratch).  If grad_dev is not NULL, writes d loss / d material into
 * grad_dev[5][grad_stride] (zero roughness gradient where clamped).  If
 * Lr_dev is not NULL, writes Lr into Lr_dev[3][lr_stride]. */
int fipt_render_loss(const fipt_shading* sh, int64_t n, int32_t n_levels,
                     const float* sigma_host, const float* material, int64_t mat_stride,
                     const float* observed, int64_t obs_stride, int32_t tonemap,
                     double* loss_dev, float* grad_dev, int64_t grad_stride,
                     float* Lr_dev, int64_t lr_stride, void* stream);

/* fipt_render_loss for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, arithmetic and results (bit for
 * bit), except that loss_dev needs room for one double only: the
 * per-workgroup partial sums go to a static array the library holds on
 * each GPU for the life of the process (FIPT_LOSS_SLOTS - 1 doubles,
 * 16 KB).  The launch never uses more partials than that (its grid is
 * capped at that many workgroups, each looping over its share of points),
 * so no n is too large; the call still returns FIPT_EINVAL with a message
 * should a launch ever need more.  The call allocates nothing (no hipMalloc
 * or hipFree, no allocating library routine).  Every call on one GPU shares
 * that array: calls that overlap on one GPU (different streams, no ordering
 * between them) race and may return a wrong loss; calls ordered on one
 * stream are safe.  The first call on each GPU looks up the array's device
 * address (FIPT_EHIP if that fails). */
int fipt_render_loss_noalloc(const fipt_shading* sh, int64_t n, int32_t n_levels,
                             const float* sigma_host, const float* material, int64_t mat_stride,
                             const float* observed, int64_t obs_stride, int32_t tonemap,
                             double* loss_dev, float* grad_dev, int64_t grad_stride,
                             float* Lr_dev, int64_t lr_stride, void* stream);

/* Emission-masked loss (Sec. 4.4, Eq. 12 and its tone-mapped form Eq. 15)
 * plus the diffuse prior (Sec. 4.5, Eq. 17), over the same inputs as
 * fipt_render_loss and an emission mask alpha[n] (device float, NULL for
 * alpha = 0 everywhere):
 *   Lhat = (1 - alpha) Lr + alpha Lgt,
 *   loss = sum over points and channels of (Gamma(Lhat) - Gamma(Lgt))^2
 *        + lambda_d * sum over points of (|1 - sigma| + |m|).
 * lambda_d must be finite and >= 0 (the paper uses 5e-4).  If grad_dev is
 * not NULL it receives d loss / d material [5][grad_stride] (the prior's
 * terms use sign(0) = 0 and are added whether or not the roughness is
 * clamped); if grad_alpha_dev is not NULL it receives d loss / d alpha [n];
 * Lr_dev, if not NULL, receives the unmasked Lr.  With alpha NULL or zero
 * and lambda_d = 0 the results equal fipt_render_loss's bit for bit.
 * loss_dev as for fipt_render_loss. */
int fipt_render_loss_masked(const fipt_shading* sh, int64_t n, int32_t n_levels,
                            const float* sigma_host, const float* material, int64_t mat_stride,
                            const float* observed, int64_t obs_stride, const float* alpha,
                            int32_t tonemap, double lambda_d, double* loss_dev, float* grad_dev,
                            int64_t grad_stride, float* grad_alpha_dev, float* Lr_dev,
                            int64_t lr_stride, void* stream);

/* out[i] = x[i] * factor_dev[0] for i < n (device float arrays, factor a
 * device double): the chain rule step of the loss's backward pass, which
 * scales the stored gradient by the incoming gradient without a host
 * round trip.  x and out may alias. */
int fipt_scale_by(const float* x, int64_t n, const double* factor_dev, float* out, void* stream);

/* ---- measurement ------------------------------------------------------- */

/* Streaming bandwidth probe: kind 0 copies c[i] = a[i], kind 1 computes the
 * triad c[i] = a[i] + s b[i], for i < n (device float arrays, 16-byte
 * aligned; b unused for a copy).  Bytes moved: 8n (copy) or 12n (triad).
 * Timed on large arrays (>= 1 GiB) it gives the HBM bandwidth a kernel can
 * reach, the reference for the memory-bound kernels besides the published
 * peak.  Asynchronous on `stream`. */
int fipt_hbm_stream(int32_t kind, const float* a, const float* b, float* c, int64_t n, float s,
                    void* stream);

/* ---- trilinear material grid (stand-in for the paper's MLP_brdf, Eq. 14) */

/* Values at n points pos[3][pos_stride] of a grid[channels][res][res][res]
 * (x fastest) whose nodes sit at bmin + (i, j, k) (bmax - bmin) / (res - 1);
 * positions are clamped onto the box.  out[channels][out_stride].
 * 2 <= res <= 1024, 1 <= channels <= 8. */
int fipt_grid_gather(const float* grid, int32_t channels, int32_t res,
                     const float* bmin_host, const float* bmax_host, const float* pos,
                     int64_t pos_stride, int64_t n, float* out, int64_t out_stride,
                     void* stream);

/* Adjoint of fipt_grid_gather for a fixed point set.  The plan sorts the
 * points once (host positions pos_host[3][n]) by node brick (8 x 8 x 8
 * nodes) and grid cell, and cuts each cell's points into columns of at most
 * 8; the adjoint sums each column in double in point order and adds the
 * column sums into the nodes as 64-bit fixed-point integers, with a scale
 * per work unit (at most 256 columns of one brick) and channel fixed by the
 * unit's largest column sum, so every node's sum is independent of the order
 * of the additions; the units of one brick are added in double in unit
 * order.  Results are bitwise reproducible.  The rounding of a column sum is
 * at most 2^-63 of (columns in its unit) x (largest column sum in the unit).
 * The plan owns device memory (20 bytes per point, 12 per column entry, 160
 * per column of the point order, 16 per unit and 32 KB per unit of a brick
 * of several).
 * 1 <= n < 2^31, 2 <= res <= 1024; FIPT_EINVAL also when the columns number
 * 2^31 or more. */
int fipt_grid_plan_create(const float* pos_host, int64_t n, int32_t res,
                          const float* bmin_host, const float* bmax_host,
                          int32_t device, fipt_grid_plan* out);
int fipt_grid_plan_destroy(fipt_grid_plan plan);

/* grad_grid[channels][res^3] = sum over points of trilinear weight times
 * grad_points[channels][gp_stride] (device), for the plan's points.
 * Overwrites grad_grid entirely; a node that a non-finite gradient reaches
 * is NaN.  Uses the plan's scratch, so calls with the same plan must not
 * overlap (one stream, or ordered streams). */
int fipt_grid_scatter(fipt_grid_plan plan, const float* grad_points, int32_t channels,
                      int64_t gp_stride, float* grad_grid, void* stream);

/* The plan's point order: order_host[q] (host, n int32) receives the index,
 * among the positions the plan was created from, of the q-th point in the
 * plan's order (by node brick, cell, then index).  Synchronous. */
int fipt_grid_plan_order(fipt_grid_plan plan, int32_t* order_host);

/* Per-point data into the plan's order: dst[c][q] = src[c][order[q]] for
 * c < planes and q < n (device float planes of the plan's n points; an
 * int32 plane can be moved as float bits).  src and dst must not overlap.
 * A set-up step: a point set whose material is fitted for many steps is put
 * into the plan's order once (shading terms, observations, or the points
 * before their bake). */
int fipt_grid_plan_permute(fipt_grid_plan plan, const float* src, int32_t planes,
                           int64_t src_stride, float* dst, int64_t dst_stride, void* stream);

/* One loss-and-gradient step of the differentiation workload, fused: for
 * the plan's n points in the plan's order (fipt_grid_plan_permute), the
 * material (a_r, a_g, a_b, sigma, m) of point q is the trilinear value of
 * grid[5][res^3] (the plan's res and box) at the plan's position q, rounded
 * to float as fipt_grid_gather stores it (the stand-in for Sigmoid(MLP_brdf)
 * of Eq. 14); Lr, the loss and d loss / d material are those of
 * fipt_render_loss (Eq. 5, Eq. 8, Eq. 2 / 15) with sh and observed in plan
 * order; grad_grid[5][res^3] receives the adjoint of the material fetch
 * applied to that gradient (the gradient as stored in float).  The material
 * and the per-point gradient equal fipt_grid_gather + fipt_render_loss on
 * the same plan-ordered inputs bit for bit; the loss is summed in a fixed
 * order over the plan order.  The adjoint sums each column (at most 8
 * points of one cell, never across a multiple of 16 points of the plan's
 * order) in single precision, weight times gradient, by a fixed segmented
 * scan, then adds the column sums into the nodes as fipt_grid_scatter does
 * (64-bit fixed point at a per-unit scale), so a node differs from
 * fipt_grid_scatter's by at most the float rounding of its column sums
 * (about 2^-21 of the sum of the absolute contributions) plus the
 * fixed-point quantum; everything is bitwise reproducible.  loss_dev holds
 * FIPT_LOSS_SLOTS doubles (the rest is scratch).  grad_points[5][gp_stride]
 * (plan order), when not NULL, also receives the per-point gradient.  Uses
 * the plan's scratch (160 bytes per column), so calls with one plan must
 * not overlap.  Allocates nothing; asynchronous on `stream`. */
int fipt_grid_render_loss(fipt_grid_plan plan, const float* grid, const fipt_shading* sh,
                          int32_t n_levels, const float* sigma_host, const float* observed,
                          int64_t obs_stride, int32_t tonemap, double* loss_dev,
                          float* grad_grid, float* grad_points, int64_t gp_stride, void* stream);

/* ---- voxel radiance cache (Sec. 4.2) ------------------------------------ */

/* Average pooling of observed pixels onto a voxel grid, the radiance cache
 * L' that Sec. 4.2 queries in Eq. 9.  The plan sorts the pixels by voxel
 * once: pos_host[3][n] (host float) are the pixels' surface points, each in
 * voxel floor((x - bmin) res / (bmax - bmin)) per axis, clamped to
 * [0, res - 1] (computed in double).  1 <= n < 2^31, 1 <= res <= 512,
 * bmin_host < bmax_host (host float [3]), finite.  The plan owns device
 * memory (4 (res^3 + 1 + n) bytes). */
int fipt_voxel_plan_create(const float* pos_host, int64_t n, int32_t res, const float* bmin_host,
                           const float* bmax_host, int32_t device, fipt_voxel_plan* out);
int fipt_voxel_plan_destroy(fipt_voxel_plan plan);

/* cache[c][v] (device float [3][cache_stride], cache_stride >= res^3) :=
 * the mean of observed[c][p] (device float [3][obs_stride], obs_stride >=
 * n) over the plan's pixels p in voxel v, summed in double in pixel order,
 * or 0 for a voxel no pixel falls in.  Every voxel is written, so results
 * are bitwise reproducible.  Asynchronous on `stream`. */
int fipt_voxel_pool(fipt_voxel_plan plan, const float* observed, int64_t obs_stride, float* cache,
                    int64_t cache_stride, void* stream);

/* ---- hash-grid material network (Eq. 14) -------------------------------- */

/* The paper's material network: (a, sigma, m) = Sigmoid(MLP(enc(x))), with
 * enc a multiresolution hash encoding of FIPT_HG_LEVELS levels, 2^19
 * entries of 2 features per level, and an MLP of two hidden layers of 64
 * with ReLU and no biases.  Level l has 16 * 2^l cells per axis over the
 * box [bmin, bmax]; a point is mapped to p = clamp((x - bmin) * inv, 0, 1)
 * with inv = 1 / (bmax - bmin) in single precision, its cell at level l is
 * c = min(floor(p N), N - 1) per axis (single precision, exact for these
 * power-of-two N), and the 8 vertices of the cell are blended trilinearly.
 * Levels 0-2 index their (N + 1)^3 vertices densely (x + y (N + 1) +
 * z (N + 1)^2); the others hash the vertex as (x ^ 2654435761 y ^
 * 805459861 z) mod 2^19 in 32-bit arithmetic.
 * params: device float [FIPT_HG_PARAMS]: tables [32][2^19][2], then W1
 * [64][64], W2 [64][64], W3 [5][64] (row = output unit).  Outputs are the
 * material planes (a_r, a_g, a_b, sigma, m), as fipt_render_loss reads them. */
#define FIPT_HG_LEVELS 32
#define FIPT_HG_LOG2_TABLE 19
#define FIPT_HG_PARAMS (32LL * (1LL << 19) * 2 + 64 * 64 + 64 * 64 + 5 * 64)

/* material[5][mat_stride] (device) for the n points pos[3][pos_stride]
 * (device).  1 <= n < 2^31; bmin_host < bmax_host (host float [3]).
 * Asynchronous on `stream`. */
int fipt_hashgrid_forward(const float* params, const float* pos, int64_t pos_stride, int64_t n,
                          const float* bmin_host, const float* bmax_host, float* material,
                          int64_t mat_stride, void* stream);

/* Floats of workspace fipt_hashgrid_backward needs for n points. */
int64_t fipt_hashgrid_workspace_floats(int64_t n);

/* Table-gradient plan of a fixed point set (device positions pos[3][pos_stride],
 * copied into the plan): for every level, each (point, corner) with a
 * nonzero trilinear weight, sorted by table slot, then point, then corner,
 * with its weight, and the slot ranges.  Built on the device on `stream`
 * (a stable radix sort per level); returns once the plan is complete.
 * 1 <= n < 2^28; bmin_host < bmax_host (host float [3]).  The plan owns
 * device memory (12 bytes per point, 8 per nonzero (point, corner) per
 * level, at most 8 per point and level, and 2 MB per level). */
int fipt_hashgrid_plan_create(const float* pos, int64_t pos_stride, int64_t n, const float* bmin_host,
                              const float* bmax_host, void* stream, fipt_hashgrid_plan* out);
int fipt_hashgrid_plan_destroy(fipt_hashgrid_plan plan);

/* Adds d(sum over points and outputs of grad_material * material) /
 * d params into grad_params (device float [FIPT_HG_PARAMS]; the caller
 * zeroes it first for a plain gradient), for the plan's points.
 * grad_material: device [5][gm_stride], gm_stride >= n.  workspace: device,
 * at least fipt_hashgrid_workspace_floats(n) floats, overwritten.  Each table
 * entry's gradient is the sum over its (point, corner) list in the plan's
 * order, in double; the weight gradients are summed in a fixed order: the
 * result is reproducible bit for bit.  A vertex of zero weight receives
 * nothing.  Calls that share a workspace must not overlap.  Asynchronous on
 * `stream`. */
int fipt_hashgrid_backward(fipt_hashgrid_plan plan, const float* params, const float* grad_material,
                           int64_t gm_stride, float* grad_params, float* workspace,
                           int64_t workspace_floats, void* stream);

/* The forward pass of a training step (Eq. 14 as in fipt_hashgrid_forward)
 * that also keeps the points' hash encoding (64 floats per point) in the
 * first 64 n floats of `workspace` (at least fipt_hashgrid_workspace_floats(n)
 * floats), and the backward pass that takes it from there instead of
 * gathering it from the tables again: fipt_hashgrid_backward_saved, called
 * with the plan of the same points, the same params and that workspace
 * untouched in between, gives fipt_hashgrid_backward's result bit for bit.
 * The material equals fipt_hashgrid_forward's bit for bit. */
int fipt_hashgrid_forward_save(const float* params, const float* pos, int64_t pos_stride, int64_t n,
                               const float* bmin_host, const float* bmax_host, float* material,
                               int64_t mat_stride, float* workspace, int64_t workspace_floats,
                               void* stream);
int fipt_hashgrid_backward_saved(fipt_hashgrid_plan plan, const float* params,
                                 const float* grad_material, int64_t gm_stride, float* grad_params,
                                 float* workspace, int64_t workspace_floats, void* stream);

/* ---- emission re-estimation (Sec. 4.4, Eq. 13) ------------------------- */

/* Under the assumption that an emitter reflects no light (f = 0), the
 * minimiser of Eq. 13 for a triangle classified as an emitter is, per
 * channel, the median of the observed values of the pixels whose primary
 * hit is that triangle.  The plan groups pixels by triangle once:
 * tri_host[n] (host) is each pixel's primary-hit triangle, -1 for none (as
 * written by fipt_gen_points), each in [-1, n_tris).  1 <= n < 2^31,
 * 1 <= n_tris < 2^31.  The plan owns device memory (4 (n + 2 n_tris + 2)
 * bytes). */
int fipt_emission_plan_create(const int32_t* tri_host, int64_t n, int64_t n_tris, int32_t device,
                              fipt_emission_plan* out);
int fipt_emission_plan_destroy(fipt_emission_plan plan);

/* le[c][t] (device float [3][le_stride]) := for every triangle t with
 * emitter[t] != 0 (device uint8 [n_tris]), the median over the pixels p of
 * t of observed[c][p] (device float [3][obs_stride]), the lower of the two
 * middle values for an even count, so the result is one of the
 * observations (negative zero is treated as zero); 0 for other triangles
 * and for triangles no pixel sees.  Exact and bitwise reproducible;
 * allocates nothing; asynchronous on `stream`.  obs_stride >= n,
 * le_stride >= n_tris.  The call lists the emitters in the plan's memory,
 * so calls with the same plan must not overlap (one stream, or ordered
 * streams). */
int fipt_emission_median(fipt_emission_plan plan, const float* observed, int64_t obs_stride,
                         const uint8_t* emitter, float* le, int64_t le_stride, void* stream);

/* ---- serving: continuous batching of bake requests --------------------- */

/* A server owns a device pool of `pool_bytes` for request outputs and a
 * scheduler thread.  Requests are admitted first come first served while
 * their output (3 + 6K planes x points x 4 bytes) fits in the pool and
 * fewer than max_inflight are admitted; admitted requests are split into
 * tiles (contiguous runs of points) placed into persistent bake launches of
 * up to samples_per_launch lobe samples: first every request whose
 * remaining work fits in one launch, whole, then the others in admission
 * order.  Requests that arrive while others run join the next launch.  Each
 * point's result is bitwise identical to fipt_bake with the same inputs. */
int fipt_server_create(int32_t device, int64_t pool_bytes, int32_t max_inflight,
                       int64_t samples_per_launch, fipt_server* out);

/* Queue a request: bake `pts` (device, borrowed until completion) of scene
 * `s` with params `p`.  Returns a ticket.  FIPT_EINVAL for invalid requests
 * or a request larger than the whole pool. */
int fipt_server_submit(fipt_server srv, fipt_scene s, const fipt_points* pts,
                       const fipt_bake_params* p, uint64_t* ticket);

/* FIPT_OK when the request completed (the result is ready), FIPT_EAGAIN
 * while pending, FIPT_ECANCELED if cancelled. */
int fipt_server_poll(fipt_server srv, uint64_t ticket);

/* Block until completion or timeout_us (< 0 = forever); FIPT_EAGAIN on
 * timeout. */
int fipt_server_wait(fipt_server srv, uint64_t ticket, int64_t timeout_us);

/* Result view of a completed request: shading planes in the server pool
 * (device), valid until fipt_server_release.  Timestamps in microseconds of
 * the server clock: submit, admit (output space granted) and completion. */
int fipt_server_result(fipt_server srv, uint64_t ticket, fipt_shading* out,
                       int64_t* t_submit_us, int64_t* t_admit_us, int64_t* t_done_us);

/* Return a completed request's pool space. */
int fipt_server_release(fipt_server srv, uint64_t ticket);

/* Cancel a queued (not yet admitted) request; FIPT_EBUSY once admitted. */
int fipt_server_cancel(fipt_server srv, uint64_t ticket);

/* Counters: launches, tiles, samples baked, requests completed, pool bytes
 * in use, requests queued (not admitted), requests in flight. */
typedef struct fipt_server_stats {
    int64_t launches;
    int64_t tiles;
    int64_t samples;
    int64_t completed;
    int64_t pool_in_use;
    int64_t queued;
    int64_t inflight;
} fipt_server_stats;
int fipt_server_stats_get(fipt_server srv, fipt_server_stats* out);

/* Stop accepting work, finish what is admitted, free the pool. */
int fipt_server_destroy(fipt_server srv);

#ifdef __cplusplus
}
#endif

#endif /* FIPT_H */
