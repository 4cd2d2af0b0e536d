// Device building blocks of the bake: counter-based random numbers,
// shading frame, lobe sampling, microfacet terms, BVH traversal and the
// radiance lookup.  Single precision throughout.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "fipt_internal.hpp"

namespace fipt {
namespace dev {

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---- Philox4x32-10 (Salmon et al., SC'11) --------------------------------
// Ten rounds; each multiplies words 0 and 2 by 0xD2511F53 / 0xCD9E8D57 and
// mixes the high halves with words 1 / 3 and the round key; the key grows
// by the Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply gives both halves of a product
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
        const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Two uniforms in [0, 1) with 24 significant bits (exact in float).
__device__ __forceinline__ void lobe_uniforms(uint64_t seed, int64_t p, int lobe, int s,
                                              float& xi1, float& xi2) {
    const uint4 c = make_uint4((uint32_t)(uint64_t)p, (uint32_t)((uint64_t)p >> 32),
                               (uint32_t)lobe, (uint32_t)s);
    const uint4 u = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    xi1 = (float)(u.x >> 8) * (1.0f / 16777216.0f);
    xi2 = (float)(u.y >> 8) * (1.0f / 16777216.0f);
}

// ---- shading frame (Duff et al., JCGT 2017), sign from n.z >= 0 ----------
__device__ __forceinline__ void make_frame(V3 n, V3& t, V3& b) {
    const float s = n.z >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (s + n.z);
    const float c = n.x * n.y * a;
    t = v3(1.0f + s * n.x * n.x * a, s * c, -s * n.x);
    b = v3(c, s + n.y * n.y * a, -n.y);
}
__device__ __forceinline__ V3 to_world(V3 t, V3 b, V3 n, float lx, float ly, float lz) {
    return v3(t.x * lx + b.x * ly + n.x * lz, t.y * lx + b.y * ly + n.y * lz,
              t.z * lx + b.z * ly + n.z * lz);
}

// Reciprocal by the hardware approximation (about 1 ulp): sampling
// directions and weights tolerate it, and a correctly rounded division
// costs ten times as many instructions.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Square root by the hardware approximation (about 1 ulp), for the same
// reason; inputs here are never denormal.
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// Smith G1 of GGX written as 2 c / (c + sqrt(alpha^2 + (1 - alpha^2) c^2)),
// c = n.v > 0 (algebraically 2 / (1 + sqrt(1 + alpha^2 tan^2))).
__device__ __forceinline__ float smith_g1(float a2, float c) {
    return 2.0f * c * rcp(c + sqrt_hw(a2 + (1.0f - a2) * c * c));
}

// ---- BVH traversal ---------------------------------------------------------
struct Hit {
    int32_t leaf;  // leaf-order triangle position, -1 on a miss
    float t, u, v;
};

// End-of-traversal marker: never a node index or a leaf reference (< 2^28
// triangles).
constexpr int32_t kDone = INT_MIN;

// Per-ray constants of the slab test: inverse direction, origin times
// inverse direction, and for each axis the byte offset inside a node of the
// near-plane vector (the low bounds when the direction component is
// positive, else the high bounds; the far-plane vector is the other one of
// the pair, 16 bytes away).
struct RaySlab {
    float ix, iy, iz, oxi, oyi, ozi;
    uint32_t nx, ny, nz;
};
__device__ __forceinline__ RaySlab ray_slab(V3 o, V3 d) {
    const float dx = fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x);
    const float dy = fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y);
    const float dz = fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z);
    RaySlab r;
    r.ix = __builtin_amdgcn_rcpf(dx);
    r.iy = __builtin_amdgcn_rcpf(dy);
    r.iz = __builtin_amdgcn_rcpf(dz);
    r.oxi = o.x * r.ix;
    r.oyi = o.y * r.iy;
    r.ozi = o.z * r.iz;
    r.nx = (__float_as_uint(r.ix) >> 31) << 4;
    r.ny = 32u + ((__float_as_uint(r.iy) >> 31) << 4);
    r.nz = 64u + ((__float_as_uint(r.iz) >> 31) << 4);
    return r;
}

// Slab test of one child box given its near and far planes, against
// [0, tmax]; returns the entry distance, or +inf when the box is missed.
// An unused slot (low bounds +inf, high bounds -inf) has near distance +inf
// and far distance -inf whatever the direction, so it is always missed.
__device__ __forceinline__ float box_entry(float nx, float fx, float ny, float fy, float nz,
                                           float fz, const RaySlab& r, float tmax) {
    const float tn = fmaxf(fmaxf(fmaf(nx, r.ix, -r.oxi), fmaf(ny, r.iy, -r.oyi)),
                           fmaxf(fmaf(nz, r.iz, -r.ozi), 0.0f));
    const float tf = fminf(fminf(fmaf(fx, r.ix, -r.oxi), fmaf(fy, r.iy, -r.oyi)),
                           fminf(fmaf(fz, r.iz, -r.ozi), tmax));
    return tn <= tf ? tn : INFINITY;
}

__device__ __forceinline__ void order2(float& ka, int32_t& ca, float& kb, int32_t& cb) {
    const bool s = kb < ka;
    const float k = s ? kb : ka;
    kb = s ? ka : kb;
    ka = k;
    const int32_t c = s ? cb : ca;
    cb = s ? ca : cb;
    ca = c;
}

// Load through a pointer known to address global memory.  Scene and point
// pointers that the serving kernel reads from a tile table are generic as far
// as the compiler can tell; loading through a global-qualified pointer gives
// global loads with a scalar base instead of flat loads (which also wait on
// the LDS counter the traversal stack uses).
// (The load goes through a native vector type: HIP's float4 is a class,
// copied through a generic pointer, which would drop the address space.)
typedef float gfloat4 __attribute__((ext_vector_type(4)));
typedef int gint4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_global(const float4* p) {
    const gfloat4 v = *(const __attribute__((address_space(1))) gfloat4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 load_global(const int4* p) {
    const gint4 v = *(const __attribute__((address_space(1))) gint4*)p;
    return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float4 node_vec(const Bvh4Node* nodes, uint32_t off) {
    return load_global(reinterpret_cast<const float4*>(reinterpret_cast<const char*>(nodes) + off));
}

// One step of closest-hit traversal at 4-wide node `ref`: the hit children
// are visited nearest first; the nearest becomes `ref`, the others are
// pushed farthest first.  With no child hit, the next entry is popped
// (kDone when the stack is empty).  Node byte offsets fit 32 bits (the
// builder rejects trees of more than kMaxNodes4 nodes).
__device__ __forceinline__ void node4_step(const Bvh4Node* nodes, int32_t& ref, int& sp,
                                           int32_t* stack, int stride, const RaySlab& r,
                                           float tmax) {
    const uint32_t base = (uint32_t)ref << 7;
    const uint32_t ox = base + r.nx, oy = base + r.ny, oz = base + r.nz;
    const float4 nx = node_vec(nodes, ox), fx = node_vec(nodes, ox ^ 16u);
    const float4 ny = node_vec(nodes, oy), fy = node_vec(nodes, oy ^ 16u);
    const float4 nz = node_vec(nodes, oz), fz = node_vec(nodes, oz ^ 16u);
    const int4 ch = load_global(reinterpret_cast<const int4*>(reinterpret_cast<const char*>(nodes) + base + 96u));
    float k0 = box_entry(nx.x, fx.x, ny.x, fy.x, nz.x, fz.x, r, tmax);
    float k1 = box_entry(nx.y, fx.y, ny.y, fy.y, nz.y, fz.y, r, tmax);
    float k2 = box_entry(nx.z, fx.z, ny.z, fy.z, nz.z, fz.z, r, tmax);
    float k3 = box_entry(nx.w, fx.w, ny.w, fy.w, nz.w, fz.w, r, tmax);
    int32_t c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
    // keep the child load in the same batch as the box loads (otherwise it
    // is sunk below the miss branch and costs a second memory round trip)
    asm volatile("" : : "v"(c0), "v"(c1), "v"(c2), "v"(c3));
    const int hits = (k0 < INFINITY) + (k1 < INFINITY) + (k2 < INFINITY) + (k3 < INFINITY);
    // sorting network on four keys
    order2(k0, c0, k1, c1);
    order2(k2, c2, k3, c3);
    order2(k0, c0, k2, c2);
    order2(k1, c1, k3, c3);
    order2(k1, c1, k2, c2);
    if (hits == 0) {
        if (sp == 0) {
            ref = kDone;
        } else {
            --sp;
            ref = stack[sp * stride];
        }
        return;
    }
    if (hits > 3) stack[(sp++) * stride] = c3;
    if (hits > 2) stack[(sp++) * stride] = c2;
    if (hits > 1) stack[(sp++) * stride] = c1;
    ref = c0;
}

// Triangle test (Moller-Trumbore) of leaf-order triangle `i`; updates the
// closest hit, exact distance ties going to the lower original index.
__device__ __forceinline__ void tri_test(const TriGeom* tris, int32_t i, V3 o, V3 d, Hit& h,
                                         int32_t& best_orig) {
    const float4* tp = reinterpret_cast<const float4*>(tris + i);
    const float4 t0 = load_global(tp);
    const float4 t1 = load_global(tp + 1);
    const float4 t2 = load_global(tp + 2);
    const V3 e1 = v3(t1.x, t1.y, t1.z);
    const V3 e2 = v3(t2.x, t2.y, t2.z);
    const V3 pv = cross(d, e2);
    const float det = dot(e1, pv);
    if (det == 0.0f) return;
    const float inv = __builtin_amdgcn_rcpf(det);
    const V3 s = o - v3(t0.x, t0.y, t0.z);
    const float u = dot(s, pv) * inv;
    const V3 q = cross(s, e1);
    const float v = dot(d, q) * inv;
    const float t = dot(e2, q) * inv;
    const int32_t orig = __float_as_int(t0.w);
    const bool inside = (u >= 0.0f) & (v >= 0.0f) & (u + v <= 1.0f) & (t > 0.0f);
    const bool nearer = (t < h.t) | ((t == h.t) & (orig < best_orig));
    if (inside & nearer) {
        h.t = t;
        h.u = u;
        h.v = v;
        h.leaf = i;
        best_orig = orig;
    }
}

// Closest hit along o + t d, t > 0, one ray per lane.  `stack` points at
// this lane's first LDS stack slot; consecutive slots are `stride` ints
// apart (lane-minor, so a wave's pushes and pops hit distinct banks).
template <bool COUNT>
__device__ __forceinline__ Hit trace(const DeviceScene& sc, V3 o, V3 d, int32_t* stack,
                                     int stride, uint32_t& n_nodes, uint32_t& n_tris) {
    const RaySlab r = ray_slab(o, d);
    Hit h;
    h.leaf = -1;
    h.t = INFINITY;
    h.u = h.v = 0.0f;
    int32_t best_orig = INT_MAX;
    int32_t ref = 0;
    int sp = 0;
    while (ref != kDone) {
        if (ref >= 0) {
            if (COUNT) ++n_nodes;
            node4_step(sc.nodes, ref, sp, stack, stride, r, h.t);
        } else {
            const int32_t lr = ~ref;
            const int32_t first = lr >> 3;
            const int32_t cnt = (lr & 7) + 1;
            for (int i = 0; i < cnt; ++i) {
                if (COUNT) ++n_tris;
                tri_test(sc.tris, first + i, o, d, h, best_orig);
            }
            if (sp == 0) {
                ref = kDone;
            } else {
                --sp;
                ref = stack[sp * stride];
            }
        }
    }
    return h;
}

// Radiance toward the ray origin at a hit: barycentric blend of the corner
// cache values plus the triangle's emission; zero on a miss.
__device__ __forceinline__ V3 radiance(const DeviceScene& sc, const Hit& h) {
    if (h.leaf < 0) return v3(0.0f, 0.0f, 0.0f);
    const float4* rp = reinterpret_cast<const float4*>(sc.rad + h.leaf);
    const float4 r0 = load_global(rp);
    const float4 r1 = load_global(rp + 1);
    const float4 r2 = load_global(rp + 2);
    const float w0 = 1.0f - h.u - h.v;
    return v3(w0 * r0.x + h.u * r0.w + h.v * r1.z + r2.y,
              w0 * r0.y + h.u * r1.x + h.v * r1.w + r2.z,
              w0 * r0.z + h.u * r1.y + h.v * r2.x + r2.w);
}

// Lanes of the wave where p holds (the wave64 ballot on a boolean; HIP's
// int-valued __ballot costs two extra instructions per call).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Sum over the 64 lanes of a wave by a fixed xor butterfly: every lane ends
// with the same, order-fixed total.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace dev
}  // namespace fipt
