// HIP kernels of the stage-3 path-traced shading refinement (Sec. 4.3,
// Eq. 10 and 11) for gfx950.
//
// Each shading integral is re-estimated by growing the stage-1 path: the
// first direction and its weight are the stage-1 lobe sample; a hit on an
// emitter returns its emission; a hit whose current roughness (trilinear
// from the material grid) exceeds the threshold, or the last allowed
// vertex, returns the radiance cache; a glossy hit continues with the full
// BRDF of Eq. 1, the radiance arriving there estimated by emitter sampling
// and BRDF sampling combined with the balance heuristic.
//
// Mapping: one wavefront per point from a persistent grid.  With at most 10
// roughness levels each lane owns one path at a time and takes the point's
// next sample when its path ends (refine_point_spec); with more, the 64
// lanes take 64 consecutive (lobe, sample) pairs and follow them to the end
// (refine_point).  Either way the lobes are summed by the fixed xor
// butterfly, so a point's result depends only on the inputs.
//
// The emitters (triangles with some channel of emission > 0, in ascending
// original index) are listed on the device at the start of each call by an
// in-order compaction: a count per block of triangles, one scan, a scatter.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "fipt_internal.hpp"

namespace fipt {
namespace {

using dev::V3;
using dev::v3;

constexpr int kBlock = 64;
constexpr int kGridWavesPerCu = 16;
constexpr int kListBlock = 256;        // triangles per block of the emitter compaction
constexpr int kScanThreads = 1024;

// ---- emitter list ------------------------------------------------------------

__device__ __forceinline__ bool emits(const TriRad& r) {
    return r.ler > 0.0f || r.leg > 0.0f || r.leb > 0.0f;
}

// Emitters among original triangles [b 256, (b + 1) 256) -> counts[b].
__global__ __launch_bounds__(kListBlock) void k_emit_count(const TriRad* rad, const int32_t* leaf_of,
                                                           int64_t T, int32_t* counts) {
    __shared__ int32_t s_w[kListBlock / 64];
    const int64_t f = (int64_t)blockIdx.x * kListBlock + threadIdx.x;
    const bool e = f < T && emits(rad[leaf_of[f]]);
    const uint64_t m = dev::ballot(e);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t c = 0;
        for (int w = 0; w < kListBlock / 64; ++w) c += s_w[w];
        counts[blockIdx.x] = c;
    }
}

// Exclusive scan of n block counts in place (one workgroup); the total goes
// to *total.
__global__ __launch_bounds__(kScanThreads) void k_emit_scan(int32_t* counts, int64_t n,
                                                            int32_t* total) {
    __shared__ int32_t s_sum[kScanThreads];
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t a = (int64_t)threadIdx.x * per, b = min(n, a + per);
    int32_t s = 0;
    for (int64_t i = a; i < b; ++i) s += counts[i];
    s_sum[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int t = 0; t < kScanThreads; ++t) {
            const int32_t v = s_sum[t];
            s_sum[t] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int32_t run = s_sum[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        const int32_t v = counts[i];
        counts[i] = run;
        run += v;
    }
}

// Each emitter's leaf position at its rank among the emitters.
__global__ __launch_bounds__(kListBlock) void k_emit_scatter(const TriRad* rad, const int32_t* leaf_of,
                                                             int64_t T, const int32_t* offsets,
                                                             int32_t* list) {
    __shared__ int32_t s_w[kListBlock / 64];
    const int64_t f = (int64_t)blockIdx.x * kListBlock + threadIdx.x;
    const int32_t leaf = f < T ? leaf_of[f] : 0;
    const bool e = f < T && emits(rad[leaf]);
    const uint64_t m = dev::ballot(e);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = __popcll(m);
    __syncthreads();
    int32_t before = offsets[blockIdx.x];
    for (int k = 0; k < w; ++k) before += s_w[k];
    if (e) list[before + __popcll(m & ((1ull << lane) - 1ull))] = leaf;
}

// ---- material, BRDF and sampling (single precision) --------------------------

struct MatGrid {
    const float* g;      // [5][R^3]
    int32_t res;
    double lo[3];
    double scale[3];     // (R - 1) / (hi - lo)
    int64_t plane;       // R^3
};

struct Material {
    float a[3], sigma, m;
};

// Trilinear value of the grid at x (vertex-aligned, clamped onto the box),
// the grid coordinates in double: the next direction of a glossy path
// depends on the roughness here, so a position error reaches the next hit
// multiplied by the roughness gradient and the path length; single-
// precision coordinates would add ~1e-7 of the box to it.
__device__ __forceinline__ Material material_at(const MatGrid& M, const double x[3]) {
    const double top = (double)(M.res - 1);
    const double ux = fmin(fmax((x[0] - M.lo[0]) * M.scale[0], 0.0), top);
    const double uy = fmin(fmax((x[1] - M.lo[1]) * M.scale[1], 0.0), top);
    const double uz = fmin(fmax((x[2] - M.lo[2]) * M.scale[2], 0.0), top);
    const int i = min((int)ux, M.res - 2), j = min((int)uy, M.res - 2), k = min((int)uz, M.res - 2);
    const float fx = (float)(ux - i), fy = (float)(uy - j), fz = (float)(uz - k);
    const int64_t R = M.res;
    const int64_t base = i + R * (j + R * (int64_t)k);
    const int64_t dy = R, dz = R * R;
    const float w000 = (1 - fx) * (1 - fy) * (1 - fz), w100 = fx * (1 - fy) * (1 - fz);
    const float w010 = (1 - fx) * fy * (1 - fz), w110 = fx * fy * (1 - fz);
    const float w001 = (1 - fx) * (1 - fy) * fz, w101 = fx * (1 - fy) * fz;
    const float w011 = (1 - fx) * fy * fz, w111 = fx * fy * fz;
    float v[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const float* G = M.g + c * M.plane + base;
        v[c] = w000 * G[0] + w100 * G[1] + w010 * G[dy] + w110 * G[dy + 1] + w001 * G[dz] +
               w101 * G[dz + 1] + w011 * G[dz + dy] + w111 * G[dz + dy + 1];
    }
    return {{v[0], v[1], v[2]}, v[3], v[4]};
}

// GGX D(h) = alpha^2 / (pi ((n.h)^2 (alpha^2 - 1) + 1)^2), its denominator
// written as |n x h|^2 + (n.h)^2 alpha^2 (unit n, h): 1 - (n.h)^2 near the
// peak of a narrow lobe is below single-precision resolution, the squared
// cross product is not.
__device__ __forceinline__ float ggx_d(float a2, V3 n, V3 h, float nh) {
    const V3 c = dev::cross(n, h);
    const float t = dev::dot(c, c) + nh * nh * a2;
    return a2 * dev::rcp(3.14159265358979f * t * t);
}

__device__ __forceinline__ V3 normalize(V3 v) { return rsqrtf(dev::dot(v, v)) * v; }

// f of Eq. 1 with the cosine: kd/pi (n.wi) + (ks F0 + F1) D G / (4 n.wo);
// zero unless both directions are above the surface.
__device__ __forceinline__ V3 brdf_f(V3 n, V3 wo, V3 wi, const Material& mt, float a2) {
    const float ci = dev::dot(n, wi), co = dev::dot(n, wo);
    if (!(ci > 0.0f) || !(co > 0.0f)) return v3(0.0f, 0.0f, 0.0f);
    const V3 h = normalize(wi + wo);
    const float nh = dev::dot(n, h), hi = dev::dot(h, wi);
    float spec = 0.0f, F1 = 0.0f;
    if (nh > 0.0f && hi > 0.0f) {
        const float G = dev::smith_g1(a2, ci) * dev::smith_g1(a2, co);
        spec = ggx_d(a2, n, h, nh) * G * dev::rcp(4.0f * co);
        const float f = 1.0f - hi, f2 = f * f;
        F1 = f2 * f2 * f;
    }
    const float m = mt.m, inv_pi = 0.318309886183791f;
    float r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float kd = mt.a[c] * (1.0f - m), ks = 0.04f * (1.0f - m) + mt.a[c] * m;
        r[c] = kd * inv_pi * ci + (ks * (1.0f - F1) + F1) * spec;
    }
    return v3(r[0], r[1], r[2]);
}

// Density of the BRDF sampling at a glossy vertex: half GGX half vectors
// (D(h)(n.h) / (4 wo.h) in wi), half cosine-weighted.
__device__ __forceinline__ float brdf_pdf(V3 n, V3 wo, V3 wi, float a2) {
    const float ci = dev::dot(n, wi);
    if (!(ci > 0.0f)) return 0.0f;
    const V3 h = normalize(wi + wo);
    const float nh = dev::dot(n, h), oh = dev::dot(wo, h);
    const float ps = (nh > 0.0f && oh > 0.0f) ? ggx_d(a2, n, h, nh) * nh * dev::rcp(4.0f * oh) : 0.0f;
    return 0.5f * ps + 0.5f * 0.318309886183791f * ci;
}

__device__ __forceinline__ float unif24(uint32_t u) { return (float)(u >> 8) * (1.0f / 16777216.0f); }

__device__ __forceinline__ uint4 vertex_philox(uint64_t seed, int64_t p, int lobe, int s, int vertex,
                                               int k) {
    const uint4 c = make_uint4((uint32_t)(uint64_t)p, (uint32_t)((uint64_t)p >> 32),
                               (uint32_t)lobe | ((uint32_t)vertex << 8) | ((uint32_t)k << 16),
                               (uint32_t)s);
    return dev::philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

struct RefineArgs {
    BakeLaunch b;
    MatGrid mat;
    float sigma_diffuse;
    int32_t max_vertices;
    int32_t nee;              // emitter sampling on
    const int32_t* emit;      // emitters' leaf positions
    const int32_t* n_emit;    // device count
};

// Unit face normal and area of leaf-order triangle i, with its first vertex.
__device__ __forceinline__ float tri_frame(const TriGeom* tris, int32_t i, V3& v0, V3& e1, V3& e2,
                                           V3& n) {
    const float4* tp = reinterpret_cast<const float4*>(tris + i);
    const float4 t0 = dev::load_global(tp), t1 = dev::load_global(tp + 1),
                 t2 = dev::load_global(tp + 2);
    v0 = v3(t0.x, t0.y, t0.z);
    e1 = v3(t1.x, t1.y, t1.z);
    e2 = v3(t2.x, t2.y, t2.z);
    const V3 c = dev::cross(e1, e2);
    const float l = sqrtf(dev::dot(c, c));
    n = (1.0f / l) * c;
    return 0.5f * l;
}

// Radiance arriving at o along d on a refined path (Eq. 10 / 11).
__device__ V3 refine_path(const RefineArgs& A, int64_t p, int lobe, int s, V3 o, V3 d,
                          int32_t* stack, int n_emit) {
    const DeviceScene& sc = A.b.sc;
    V3 T = v3(1.0f, 1.0f, 1.0f), C = v3(0.0f, 0.0f, 0.0f);
    float pb_prev = -1.0f;
    const bool nee = A.nee && n_emit > 0;
    uint32_t z0 = 0, z1 = 0;
    for (int vert = 1;; ++vert) {
        const dev::Hit h = dev::trace<false>(sc, o, d, stack, kBlock, z0, z1);
        if (h.leaf < 0) break;
        const float4 r2 = dev::load_global(reinterpret_cast<const float4*>(sc.rad + h.leaf) + 2);
        if (r2.y > 0.0f || r2.z > 0.0f || r2.w > 0.0f) {
            // an emitter: its emission, weighted against emitter sampling
            float w = 1.0f;
            if (pb_prev >= 0.0f && nee) {
                V3 v0, e1, e2, nz;
                const float area = tri_frame(sc.tris, h.leaf, v0, e1, e2, nz);
                const float cz = fabsf(dev::dot(nz, d));
                // (cz = 0 gives pl = inf and w = 0, as a grazing hit has no
                // emitter-sampling density to compete with)
                const float pl = h.t * h.t * dev::rcp(cz * (float)n_emit * area);
                w = pb_prev * dev::rcp(pb_prev + pl);
            }
            C = C + v3(T.x * r2.y * w, T.y * r2.z * w, T.z * r2.w * w);
            break;
        }
        // the hit point from its barycentric weights, in double (an error of
        // o + t d in single precision is ~1e-7 of the ray's length; the
        // weights place it within ~1e-7 of the triangle's edges)
        V3 v0, e1, e2, ny;
        tri_frame(sc.tris, h.leaf, v0, e1, e2, ny);
        const double yd[3] = {(double)v0.x + (double)h.u * e1.x + (double)h.v * e2.x,
                              (double)v0.y + (double)h.u * e1.y + (double)h.v * e2.y,
                              (double)v0.z + (double)h.u * e1.z + (double)h.v * e2.z};
        const V3 y = v3((float)yd[0], (float)yd[1], (float)yd[2]);
        const V3 wo = v3(-d.x, -d.y, -d.z);
        if (dev::dot(ny, wo) < 0.0f) ny = v3(-ny.x, -ny.y, -ny.z);
        if (!(dev::dot(ny, wo) > 0.0f)) break;
        const Material mt = material_at(A.mat, yd);
        if (mt.sigma > A.sigma_diffuse || vert >= A.max_vertices) {
            const V3 R = dev::radiance(sc, h);   // cache only: no emission here
            C = C + v3(T.x * R.x, T.y * R.y, T.z * R.z);
            break;
        }
        // a glossy vertex: the BRDF of the current material
        const float sg = fminf(fmaxf(mt.sigma, 0.02f), 1.0f);
        const float alpha = sg * sg, a2 = alpha * alpha;
        const V3 yo = y + A.b.eps * ny;
        const uint4 u = vertex_philox(A.b.seed, p, lobe, s, vert, 0);
        const uint4 vv = vertex_philox(A.b.seed, p, lobe, s, vert, 1);
        if (nee) {
            const int32_t fe = A.emit[__umulhi(u.x, (uint32_t)n_emit)];
            V3 q0, q1, q2, nz;
            const float area = tri_frame(sc.tris, fe, q0, q1, q2, nz);
            const float su = dev::sqrt_hw(unif24(u.y)), xb = unif24(u.z);
            const V3 z = q0 + (su * (1.0f - xb)) * q1 + (su * xb) * q2;
            V3 l = z - yo;
            const float dist = sqrtf(dev::dot(l, l));
            l = (1.0f / dist) * l;
            const float cz = fabsf(dev::dot(nz, l));
            if (dev::dot(ny, l) > 0.0f && cz > 0.0f) {
                const dev::Hit sh = dev::trace<false>(sc, yo, l, stack, kBlock, z0, z1);
                if (sh.leaf == fe) {
                    const V3 fv = brdf_f(ny, wo, l, mt, a2);
                    const float pl = dist * dist * dev::rcp(cz * (float)n_emit * area);
                    const float inv = dev::rcp(pl + brdf_pdf(ny, wo, l, a2));
                    const float4 e = dev::load_global(reinterpret_cast<const float4*>(sc.rad + fe) + 2);
                    C = C + v3(T.x * fv.x * e.y * inv, T.y * fv.y * e.z * inv, T.z * fv.z * e.w * inv);
                }
            }
        }
        // continue along a direction drawn from f, in the frame of the hit
        // triangle's first edge (t = e1 / |e1|, b = n x t): no sign decision
        // on n, whose single-precision components may sit a hair from zero
        // where the exact normal has a zero component
        const V3 ft = normalize(e1);
        const V3 fb = dev::cross(ny, ft);
        const float xi1 = unif24(vv.x), xi2 = unif24(vv.y);
        float sp_, cp_;
        sp_ = __builtin_amdgcn_sinf(xi2);   // sin, cos of 2 pi xi2 (angle in turns)
        cp_ = __builtin_amdgcn_cosf(xi2);
        V3 w2;
        if (unif24(u.w) < 0.5f) {
            const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
            const float cos_m = dev::rsq_ge1(1.0f + tan2);
            const float sin_m = dev::sqrt_hw(tan2) * cos_m;
            const V3 m = dev::to_world(ft, fb, ny, sin_m * cp_, sin_m * sp_, cos_m);
            const float om = dev::dot(wo, m);
            if (!(om > 0.0f)) break;
            w2 = (2.0f * om) * m - wo;
        } else {
            const float r = dev::sqrt_hw(xi1);
            w2 = dev::to_world(ft, fb, ny, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
        }
        if (!(dev::dot(ny, w2) > 0.0f)) break;
        const float pb = brdf_pdf(ny, wo, w2, a2);
        if (!(pb > 0.0f)) break;
        const V3 fv = brdf_f(ny, wo, w2, mt, a2);
        const float ipb = dev::rcp(pb);
        T = v3(T.x * fv.x * ipb, T.y * fv.y * ipb, T.z * fv.z * ipb);
        o = yo;
        d = w2;
        pb_prev = pb;
    }
    return C;
}

// Refine point p with the calling wavefront (the chunked bake's layout).
__device__ void refine_point(const RefineArgs& A, int64_t p, int lane, int32_t* stack, int n_emit) {
    const BakeLaunch& b = A.b;
    const int K = b.K;
    const int P = 3 + 6 * K;
    const int64_t ps = b.pts_stride;
    const int32_t tri = b.ptri[p];
    V3 x = v3(b.pts[p], b.pts[ps + p], b.pts[2 * ps + p]);
    V3 n = v3(b.pts[3 * ps + p], b.pts[4 * ps + p], b.pts[5 * ps + p]);
    const V3 wo = v3(b.pts[6 * ps + p], b.pts[7 * ps + p], b.pts[8 * ps + p]);
    float cos_o = dev::dot(n, wo);
    if (tri >= 0 && cos_o < 0.0f) {
        n = v3(-n.x, -n.y, -n.z);
        cos_o = -cos_o;
    }
    const int64_t os = b.out_stride;
    if (!(tri >= 0 && cos_o > 0.0f)) {
        for (int j = lane; j < P; j += 64) b.out[(int64_t)j * os + p] = 0.0f;
        return;
    }
    V3 ft, fb;
    dev::make_frame(n, ft, fb);
    const V3 o = x + b.eps * n;
    const int64_t rng_p = p + b.p_offset;
    const int spp_d = b.spp_d, spp_s = b.spp_s;
    const int S = spp_d + K * spp_s;
    float acc_a = 0.0f, acc_b = 0.0f;
    for (int q0 = 0; q0 < S; q0 += 64) {
        const int q = q0 + lane;
        const bool active = q < S;
        const int lobe = active ? dev::lobe_of(q, spp_d, spp_s) : -1;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f, c4 = 0.0f, c5 = 0.0f;
        if (active) {
            const int s = lobe == 0 ? q : (q - spp_d) - (lobe - 1) * spp_s;
            float xi1, xi2;
            dev::lobe_uniforms(b.seed, rng_p, lobe, s, lobe == 0 ? b.w_d : b.w_s, xi1, xi2);
            float sp_, cp_;
            sp_ = __builtin_amdgcn_sinf(xi2);   // sin, cos of 2 pi xi2 (angle in turns)
            cp_ = __builtin_amdgcn_cosf(xi2);
            V3 wi = v3(0.0f, 0.0f, 1.0f);
            float w = 0.0f, F1 = 0.0f;
            bool shoot = false;
            if (lobe == 0) {
                const float r = dev::sqrt_hw(xi1);
                wi = dev::to_world(ft, fb, n, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
                w = 1.0f;
                shoot = true;
            } else {
                const float sg = b.sigma[lobe - 1];
                const float alpha = sg * sg;
                const float a2 = alpha * alpha;
                const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
                const float cos_m = dev::rsq_ge1(1.0f + tan2);
                const float sin_m = dev::sqrt_hw(tan2) * cos_m;
                const V3 m = dev::to_world(ft, fb, n, sin_m * cp_, sin_m * sp_, cos_m);
                const float om = dev::dot(wo, m);
                if (om > 0.0f) {
                    wi = (2.0f * om) * m - wo;
                    const float ci = dev::dot(n, wi);
                    if (ci > 0.0f) {
                        const float G = dev::smith_g1(a2, ci) * dev::smith_g1(a2, cos_o);
                        w = G * om * dev::rcp(cos_o * cos_m);
                        const float f = 1.0f - om;
                        const float f2 = f * f;
                        F1 = f2 * f2 * f;
                        shoot = true;
                    }
                }
            }
            if (shoot) {
                const V3 R = refine_path(A, rng_p, lobe, s, o, wi, stack, n_emit);
                if (lobe == 0) {
                    c0 = R.x;
                    c1 = R.y;
                    c2 = R.z;
                } else {
                    const float w0 = w * (1.0f - F1), w1 = w * F1;
                    c0 = R.x * w0;
                    c1 = R.y * w0;
                    c2 = R.z * w0;
                    c3 = R.x * w1;
                    c4 = R.y * w1;
                    c5 = R.z * w1;
                }
            }
        }
        const int l_first = dev::lobe_of(q0, spp_d, spp_s);
        const int l_last = dev::lobe_of(min(q0 + 63, S - 1), spp_d, spp_s);
        for (int l = l_first; l <= l_last; ++l) {
            const bool mine = lobe == l;
            const float r0 = dev::wave_sum(mine ? c0 : 0.0f);
            const float r1 = dev::wave_sum(mine ? c1 : 0.0f);
            const float r2 = dev::wave_sum(mine ? c2 : 0.0f);
            const int base = l == 0 ? 0 : 3 + 6 * (l - 1);
            float r3 = 0.0f, r4 = 0.0f, r5 = 0.0f;
            if (l > 0) {
                r3 = dev::wave_sum(mine ? c3 : 0.0f);
                r4 = dev::wave_sum(mine ? c4 : 0.0f);
                r5 = dev::wave_sum(mine ? c5 : 0.0f);
            }
            const int na = lane - base, nb = lane + 64 - base;
            const float ra = na == 0 ? r0 : na == 1 ? r1 : na == 2 ? r2 : na == 3 ? r3 : na == 4 ? r4 : r5;
            const float rb = nb == 0 ? r0 : nb == 1 ? r1 : nb == 2 ? r2 : nb == 3 ? r3 : nb == 4 ? r4 : r5;
            const int width = l == 0 ? 3 : 6;
            if (na >= 0 && na < width) acc_a += ra;
            if (nb >= 0 && nb < width) acc_b += rb;
        }
    }
    if (lane < P) {
        const float cnt = lane < 3 ? (float)spp_d : (float)spp_s;
        b.out[(int64_t)dev::slot_plane(lane, K) * os + p] = acc_a / cnt;
    }
    if (64 + lane < P) b.out[(int64_t)dev::slot_plane(64 + lane, K) * os + p] = acc_b / (float)spp_s;
}

// Refine point p with the calling wavefront, each lane owning one path at a
// time (the refill bake's layout).  The busy lanes walk the tree together in
// the bake's node loop with speculative leaf parking; a ray is a path segment
// or the shadow ray of a glossy vertex's emitter sample.  Lanes whose ray has
// ended take their next ray together once kHitMin of them wait (or no ray is
// in flight); a lane whose path has ended adds its radiance into its current
// lobe's sums, and once kRefillMin lanes are free they take the next samples
// of the point in lane order (a ballot), so the schedule, and the result,
// depend only on the inputs.  Each path's arithmetic and random numbers are
// those of refine_path.
constexpr int kRefillMin = 40;
constexpr int kRefillMaxK = 10;
constexpr int kHitMin = 16;        // ended rays processed together once this many wait
constexpr int kSearchMin = 8;      // leave the node loop below this many searchers
enum PathState { kIdle = 0, kTracing = 1, kFinished = 2, kHit = 3 };

// A leaf reference: negative but not kDone (INT_MIN).
__device__ __forceinline__ bool is_leaf(int32_t ref) { return (uint32_t)ref > (uint32_t)dev::kDone; }
using dev::kDone;

__device__ void refine_point_spec(const RefineArgs& A, int64_t p, int lane, int32_t* stack, int n_emit) {
    const BakeLaunch& b = A.b;
    const DeviceScene& sc = b.sc;
    const int K = b.K;
    const int P = 3 + 6 * K;
    const int64_t ps = b.pts_stride;
    const int32_t tri = b.ptri[p];
    V3 x = v3(b.pts[p], b.pts[ps + p], b.pts[2 * ps + p]);
    V3 n = v3(b.pts[3 * ps + p], b.pts[4 * ps + p], b.pts[5 * ps + p]);
    const V3 wo0 = v3(b.pts[6 * ps + p], b.pts[7 * ps + p], b.pts[8 * ps + p]);
    float cos_o = dev::dot(n, wo0);
    if (tri >= 0 && cos_o < 0.0f) {
        n = v3(-n.x, -n.y, -n.z);
        cos_o = -cos_o;
    }
    const int64_t os = b.out_stride;
    if (!(tri >= 0 && cos_o > 0.0f)) {
        for (int j = lane; j < P; j += 64) b.out[(int64_t)j * os + p] = 0.0f;
        return;
    }
    V3 pft, pfb;
    dev::make_frame(n, pft, pfb);
    const V3 o0 = x + b.eps * n;
    const int64_t rng_p = p + b.p_offset;
    const int spp_d = b.spp_d, spp_s = b.spp_s;
    const int S = spp_d + K * spp_s;
    const bool nee = A.nee && n_emit > 0;

    // output slot j belongs to lane j; lobe sums flushed as in the refill bake
    float own = 0.0f;
    float cur0 = 0.0f, cur1 = 0.0f, cur2 = 0.0f, cur3 = 0.0f, cur4 = 0.0f, cur5 = 0.0f;
    int cur_lobe = -1;
    auto flush = [&](bool need) {
        uint64_t m = dev::ballot(need);
        while (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int l = __shfl(cur_lobe, leader, 64);
            const bool in = need && cur_lobe == l;
            m &= ~dev::ballot(in);
            const float s0 = dev::wave_sum(in ? cur0 : 0.0f);
            const float s1 = dev::wave_sum(in ? cur1 : 0.0f);
            const float s2 = dev::wave_sum(in ? cur2 : 0.0f);
            float s3 = 0.0f, s4 = 0.0f, s5 = 0.0f;
            if (l > 0) {
                s3 = dev::wave_sum(in ? cur3 : 0.0f);
                s4 = dev::wave_sum(in ? cur4 : 0.0f);
                s5 = dev::wave_sum(in ? cur5 : 0.0f);
            }
            const int r = lane - (l == 0 ? 0 : 3 + 6 * (l - 1));
            if (r >= 0 && r < (l == 0 ? 3 : 6))
                own += r == 0 ? s0 : r == 1 ? s1 : r == 2 ? s2 : r == 3 ? s3 : r == 4 ? s4 : s5;
        }
    };

    int state = kIdle;
    int lobe = 0, s = 0;
    float w0 = 0.0f, w1 = 0.0f;
    // the path: the ray to trace, throughput, radiance so far, the density
    // of the BRDF sample that led here (-1 for the stage-1 sample), vertex
    V3 o = o0, d = v3(0.0f, 0.0f, 1.0f), T = v3(1.0f, 1.0f, 1.0f), C = v3(0.0f, 0.0f, 0.0f);
    float pb_prev = -1.0f;
    int vert = 1;
    // a shadow ray in flight: its emitter and what it adds when unoccluded;
    // then the continuation (valid or not)
    bool shadow = false;
    int32_t fe = -1;
    V3 cn = v3(0.0f, 0.0f, 0.0f);
    bool cont = false;
    V3 o2 = o0, d2 = d, T2 = T;
    float pb2 = 0.0f;
    int next_q = 0;

    // traversal state of the lane's ray
    int32_t ref = kDone;
    int32_t* top = stack;
    dev::RaySlab rs = dev::ray_slab(o, d, sc.box_scale);
    dev::Hit h;
    h.leaf = -1;
    h.t = dev::kNoHit;
    h.u = h.v = 0.0f;
    int32_t best_orig = INT_MAX;
    auto start_ray = [&]() {
        rs = dev::ray_slab(o, d, sc.box_scale);
        ref = 0;
        top = stack;
        h.leaf = -1;
        h.t = dev::kNoHit;
        h.u = h.v = 0.0f;
        best_orig = INT_MAX;
        state = kTracing;
    };
    // what a lane does with its ended ray: the next ray of its path
    // (start_ray) or the end of the path (kFinished)
    auto process_hit = [&]() {
        if (shadow) {
            if (h.leaf == fe) C = C + cn;
            shadow = false;
            if (cont) {
                o = o2;
                d = d2;
                T = T2;
                pb_prev = pb2;
                ++vert;
                start_ray();
            } else {
                state = kFinished;
            }
            return;
        }
        if (h.leaf < 0) {
            state = kFinished;
            return;
        }
        const float4 r2 = dev::load_global(reinterpret_cast<const float4*>(sc.rad + h.leaf) + 2);
        if (r2.y > 0.0f || r2.z > 0.0f || r2.w > 0.0f) {
            float w = 1.0f;
            if (pb_prev >= 0.0f && nee) {
                V3 v0, e1, e2, nz;
                const float area = tri_frame(sc.tris, h.leaf, v0, e1, e2, nz);
                const float cz = fabsf(dev::dot(nz, d));
                const float pl = h.t * h.t * dev::rcp(cz * (float)n_emit * area);
                w = pb_prev * dev::rcp(pb_prev + pl);
            }
            C = C + v3(T.x * r2.y * w, T.y * r2.z * w, T.z * r2.w * w);
            state = kFinished;
            return;
        }
        V3 v0, e1, e2, ny;
        tri_frame(sc.tris, h.leaf, v0, e1, e2, ny);
        const double yd[3] = {(double)v0.x + (double)h.u * e1.x + (double)h.v * e2.x,
                              (double)v0.y + (double)h.u * e1.y + (double)h.v * e2.y,
                              (double)v0.z + (double)h.u * e1.z + (double)h.v * e2.z};
        const V3 y = v3((float)yd[0], (float)yd[1], (float)yd[2]);
        const V3 wo = v3(-d.x, -d.y, -d.z);
        if (dev::dot(ny, wo) < 0.0f) ny = v3(-ny.x, -ny.y, -ny.z);
        if (!(dev::dot(ny, wo) > 0.0f)) {
            state = kFinished;
            return;
        }
        const Material mt = material_at(A.mat, yd);
        if (mt.sigma > A.sigma_diffuse || vert >= A.max_vertices) {
            const V3 R = dev::radiance(sc, h);
            C = C + v3(T.x * R.x, T.y * R.y, T.z * R.z);
            state = kFinished;
            return;
        }
        const float sg = fminf(fmaxf(mt.sigma, 0.02f), 1.0f);
        const float alpha = sg * sg, a2 = alpha * alpha;
        const V3 yo = y + b.eps * ny;
        const uint4 u = vertex_philox(b.seed, rng_p, lobe, s, vert, 0);
        const uint4 vv = vertex_philox(b.seed, rng_p, lobe, s, vert, 1);
        bool shoot_shadow = false;
        V3 l = v3(0.0f, 0.0f, 1.0f);
        if (nee) {
            fe = A.emit[__umulhi(u.x, (uint32_t)n_emit)];
            V3 q0, q1, q2, nz;
            const float area = tri_frame(sc.tris, fe, q0, q1, q2, nz);
            const float su = dev::sqrt_hw(unif24(u.y)), xb = unif24(u.z);
            const V3 z = q0 + (su * (1.0f - xb)) * q1 + (su * xb) * q2;
            l = z - yo;
            const float dist = sqrtf(dev::dot(l, l));
            l = (1.0f / dist) * l;
            const float cz = fabsf(dev::dot(nz, l));
            if (dev::dot(ny, l) > 0.0f && cz > 0.0f) {
                const V3 fv = brdf_f(ny, wo, l, mt, a2);
                const float pl = dist * dist * dev::rcp(cz * (float)n_emit * area);
                const float inv = dev::rcp(pl + brdf_pdf(ny, wo, l, a2));
                const float4 e = dev::load_global(reinterpret_cast<const float4*>(sc.rad + fe) + 2);
                cn = v3(T.x * fv.x * e.y * inv, T.y * fv.y * e.z * inv, T.z * fv.z * e.w * inv);
                shoot_shadow = true;
            }
        }
        const V3 ft = normalize(e1);
        const V3 fb = dev::cross(ny, ft);
        const float xi1 = unif24(vv.x), xi2 = unif24(vv.y);
        float sp_, cp_;
        sp_ = __builtin_amdgcn_sinf(xi2);   // sin, cos of 2 pi xi2 (angle in turns)
        cp_ = __builtin_amdgcn_cosf(xi2);
        V3 w2 = v3(0.0f, 0.0f, 0.0f);
        cont = true;
        if (unif24(u.w) < 0.5f) {
            const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
            const float cos_m = dev::rsq_ge1(1.0f + tan2);
            const float sin_m = dev::sqrt_hw(tan2) * cos_m;
            const V3 m = dev::to_world(ft, fb, ny, sin_m * cp_, sin_m * sp_, cos_m);
            const float om = dev::dot(wo, m);
            if (!(om > 0.0f)) cont = false;
            else w2 = (2.0f * om) * m - wo;
        } else {
            const float r = dev::sqrt_hw(xi1);
            w2 = dev::to_world(ft, fb, ny, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
        }
        float pb = 0.0f;
        if (cont && !(dev::dot(ny, w2) > 0.0f)) cont = false;
        if (cont) {
            pb = brdf_pdf(ny, wo, w2, a2);
            if (!(pb > 0.0f)) cont = false;
        }
        if (cont) {
            const V3 fv = brdf_f(ny, wo, w2, mt, a2);
            const float ipb = dev::rcp(pb);
            T2 = v3(T.x * fv.x * ipb, T.y * fv.y * ipb, T.z * fv.z * ipb);
            o2 = yo;
            d2 = w2;
            pb2 = pb;
        }
        if (shoot_shadow) {
            o = yo;
            d = l;
            shadow = true;
            start_ray();
        } else if (cont) {
            o = o2;
            d = d2;
            T = T2;
            pb_prev = pb2;
            ++vert;
            start_ray();
        } else {
            state = kFinished;
        }
    };

    while (true) {
        // ---- lanes whose ray has ended take their next ray, together --------
        uint64_t tracing = dev::ballot(state == kTracing);
        const uint64_t ended = dev::ballot(state == kHit);
        if (ended != 0 && (__popcll(ended) >= kHitMin || tracing == 0)) {
            if (state == kHit) process_hit();
            tracing = dev::ballot(state == kTracing);
        }
        // ---- fold finished paths and refill free lanes -----------------------
        const uint64_t busy = tracing | dev::ballot(state == kHit);
        const int n_free = 64 - __popcll(busy);
        if ((n_free >= kRefillMin && next_q < S) || busy == 0) {
            const bool done = state == kFinished;
            flush(done && cur_lobe >= 0 && cur_lobe != lobe);
            if (done) {
                if (cur_lobe != lobe) {
                    cur0 = cur1 = cur2 = cur3 = cur4 = cur5 = 0.0f;
                    cur_lobe = lobe;
                }
                cur0 += C.x * w0;
                cur1 += C.y * w0;
                cur2 += C.z * w0;
                cur3 += C.x * w1;
                cur4 += C.y * w1;
                cur5 += C.z * w1;
                state = kIdle;
            }
            if (next_q >= S && busy == 0) break;
            if (next_q < S) {
                if (state == kIdle) {
                    const int rank = __popcll(~busy & ((1ull << lane) - 1ull));
                    const int q = next_q + rank;
                    if (q < S) {
                        lobe = dev::lobe_of(q, spp_d, spp_s);
                        s = lobe == 0 ? q : (q - spp_d) - (lobe - 1) * spp_s;
                        float xi1, xi2;
                        dev::lobe_uniforms(b.seed, rng_p, lobe, s, lobe == 0 ? b.w_d : b.w_s, xi1, xi2);
                        float sp_, cp_;
                        sp_ = __builtin_amdgcn_sinf(xi2);   // sin, cos of 2 pi xi2 (angle in turns)
                        cp_ = __builtin_amdgcn_cosf(xi2);
                        bool shoot = false;
                        if (lobe == 0) {
                            const float r = dev::sqrt_hw(xi1);
                            d = dev::to_world(pft, pfb, n, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
                            w0 = 1.0f;
                            w1 = 0.0f;
                            shoot = true;
                        } else {
                            const float sg = b.sigma[lobe - 1];
                            const float alpha = sg * sg;
                            const float a2 = alpha * alpha;
                            const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
                            const float cos_m = dev::rsq_ge1(1.0f + tan2);
                            const float sin_m = dev::sqrt_hw(tan2) * cos_m;
                            const V3 m = dev::to_world(pft, pfb, n, sin_m * cp_, sin_m * sp_, cos_m);
                            const float om = dev::dot(wo0, m);
                            if (om > 0.0f) {
                                d = (2.0f * om) * m - wo0;
                                const float ci = dev::dot(n, d);
                                if (ci > 0.0f) {
                                    const float G = dev::smith_g1(a2, ci) * dev::smith_g1(a2, cos_o);
                                    const float w = G * om * dev::rcp(cos_o * cos_m);
                                    const float f = 1.0f - om;
                                    const float f2 = f * f;
                                    const float F1 = f2 * f2 * f;
                                    w0 = w * (1.0f - F1);
                                    w1 = w * F1;
                                    shoot = true;
                                }
                            }
                        }
                        if (shoot) {
                            o = o0;
                            T = v3(1.0f, 1.0f, 1.0f);
                            C = v3(0.0f, 0.0f, 0.0f);
                            pb_prev = -1.0f;
                            vert = 1;
                            shadow = false;
                            start_ray();
                        }
                    }
                }
                next_q = min(S, next_q + n_free);
            }
        }
        // ---- traversal: inner nodes until every lane has parked a leaf ----
        // (lanes not tracing hold ref == kDone)
        int32_t pend = kDone;
        const uint64_t wave = dev::ballot(true);
        while (true) {
            // (the lanes left without a parked leaf are taken from the two
            // compares before the branch, so the masks stay scalar)
            const bool waits = pend == kDone;
            const bool leaf = is_leaf(ref);
            const uint64_t unparked = dev::ballot(waits) & ~dev::ballot(leaf);
            if (waits && leaf) {
                pend = ref;
                dev::stack_pop(ref, top, stack, kBlock);
            }
            const bool inner = ref >= 0;
            const uint64_t searching = dev::ballot(inner) & unparked;
            const int n_searching = __builtin_popcount((uint32_t)searching) +
                                    __builtin_popcount((uint32_t)(searching >> 32));
            if (searching == 0 || (n_searching < kSearchMin && (wave & ~unparked) != 0)) break;
            if (inner) dev::node4_step(sc.nodes, ref, top, stack, kBlock, rs, h.t);
        }
        if (pend != kDone) {
            const int32_t lr = ~pend;
            const int32_t first = lr >> 3;
            const int32_t cnt = (lr & 7) + 1;
            for (int k = 0; k < cnt; ++k) dev::tri_test(sc.tris, first + k, o, d, h, best_orig);
        }
        if (state == kTracing && ref == kDone) state = kHit;
    }
    flush(cur_lobe >= 0);
    if (lane < P) {
        const float cnt = lane < 3 ? (float)spp_d : (float)spp_s;
        b.out[(int64_t)dev::slot_plane(lane, K) * os + p] = own / cnt;
    }
}

// The chunked layout (any K) or the per-lane paths (K <= kRefillMaxK), one
// instance each, so that each gets its own register allocation.
template <bool CHUNKED>
__global__ __launch_bounds__(kBlock) void k_refine(RefineArgs A, int32_t* counters) {
    __shared__ int32_t s_stack[kStackSize * kBlock];
    const int lane = threadIdx.x & 63;
    int32_t* stack = s_stack + threadIdx.x;
    const int n_emit = __builtin_amdgcn_readfirstlane(*A.n_emit);
    const int home = (int)(blockIdx.x % kXcdCount);
    int tried = 0;
    for (int64_t p; (p = dev::next_point(counters, home, tried, A.b.n, lane)) >= 0;) {
        if (CHUNKED) refine_point(A, p, lane, stack, n_emit);
        else refine_point_spec(A, p, lane, stack, n_emit);
    }
}

__global__ void k_zero_counters_r(int32_t* counters) {
    if (threadIdx.x < kXcdCount) counters[threadIdx.x] = 0;
}

int check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

}  // namespace

int launch_emitter_list(const TriRad* rad, const int32_t* leaf_of, int64_t n_tris, int32_t* blocks,
                        int32_t* list, int32_t* count, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = (n_tris + kListBlock - 1) / kListBlock;
    hipLaunchKernelGGL(k_emit_count, dim3((unsigned)nb), dim3(kListBlock), 0, st, rad, leaf_of, n_tris,
                       blocks);
    hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(kScanThreads), 0, st, blocks, nb, count);
    hipLaunchKernelGGL(k_emit_scatter, dim3((unsigned)nb), dim3(kListBlock), 0, st, rad, leaf_of,
                       n_tris, blocks, list);
    return check("emitter list");
}

int launch_refine(const BakeLaunch& b, const RefineLaunch& r, int32_t* counters, void* stream) {
    RefineArgs A;
    A.b = b;
    A.mat.g = r.grid;
    A.mat.res = r.res;
    A.mat.plane = (int64_t)r.res * r.res * r.res;
    for (int k = 0; k < 3; ++k) {
        A.mat.lo[k] = r.bmin[k];
        A.mat.scale[k] = (double)(r.res - 1) / ((double)r.bmax[k] - (double)r.bmin[k]);
    }
    A.sigma_diffuse = r.sigma_diffuse;
    A.max_vertices = r.max_vertices;
    A.nee = (r.flags & FIPT_REFINE_BSDF_ONLY) ? 0 : 1;
    A.emit = r.emit;
    A.n_emit = r.n_emit;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t blocks = std::min<int64_t>(b.n, (int64_t)cus * kGridWavesPerCu);
    blocks = std::max<int64_t>(kXcdCount, (blocks + kXcdCount - 1) / kXcdCount * kXcdCount);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_counters_r, dim3(1), dim3(64), 0, st, counters);
    // the per-lane paths give every output slot its own lane (3 + 6K <= 64)
    if (A.b.K <= kRefillMaxK)
        hipLaunchKernelGGL(k_refine<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, A, counters);
    else
        hipLaunchKernelGGL(k_refine<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, A, counters);
    return check("refine");
}

}  // namespace fipt
