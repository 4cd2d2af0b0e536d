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
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
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

// Smith G1 of GGX written as 2 c / (c + sqrt(alpha^2 + (1 - alpha^2) c^2)),
// c = n.v > 0 (algebraically 2 / (1 + sqrt(1 + alpha^2 tan^2))).
__device__ __forceinline__ float smith_g1(float a2, float c) {
    return 2.0f * c / (c + sqrtf(a2 + (1.0f - a2) * c * c));
}

// ---- BVH traversal ---------------------------------------------------------
struct Hit {
    int32_t leaf;  // leaf-order triangle position, -1 on a miss
    float t, u, v;
};

// Closest hit along o + t d, t > 0.  `stack` points at this lane's first
// LDS stack slot; consecutive slots are `stride` ints apart (lane-minor, so
// a wave's pushes and pops hit distinct banks).  Exact distance ties go to
// the lower original triangle index.
template <bool COUNT>
__device__ __forceinline__ Hit trace(const DeviceScene& sc, V3 o, V3 d, int32_t* stack,
                                     int stride, uint32_t& n_nodes, uint32_t& n_tris) {
    const float dx = fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x);
    const float dy = fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y);
    const float dz = fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z);
    const float ix = __builtin_amdgcn_rcpf(dx), iy = __builtin_amdgcn_rcpf(dy),
                iz = __builtin_amdgcn_rcpf(dz);
    const float ox = o.x * ix, oy = o.y * iy, oz = o.z * iz;
    Hit h;
    h.leaf = -1;
    h.t = INFINITY;
    h.u = h.v = 0.0f;
    int32_t best_orig = INT_MAX;
    int32_t ref = 0;
    int sp = 0;
    while (true) {
        if (ref >= 0) {
            if (COUNT) ++n_nodes;
            const float4* np = reinterpret_cast<const float4*>(sc.nodes + ref);
            const float4 a = np[0];
            const float4 b = np[1];
            const float4 c = np[2];
            const int4 cc = reinterpret_cast<const int4*>(np)[3];
            const float a_lx = fmaf(a.x, ix, -ox), a_hx = fmaf(a.y, ix, -ox);
            const float a_ly = fmaf(a.z, iy, -oy), a_hy = fmaf(a.w, iy, -oy);
            const float a_lz = fmaf(c.x, iz, -oz), a_hz = fmaf(c.y, iz, -oz);
            const float b_lx = fmaf(b.x, ix, -ox), b_hx = fmaf(b.y, ix, -ox);
            const float b_ly = fmaf(b.z, iy, -oy), b_hy = fmaf(b.w, iy, -oy);
            const float b_lz = fmaf(c.z, iz, -oz), b_hz = fmaf(c.w, iz, -oz);
            const float tmin0 = fmaxf(fmaxf(fminf(a_lx, a_hx), fminf(a_ly, a_hy)),
                                      fmaxf(fminf(a_lz, a_hz), 0.0f));
            const float tmax0 = fminf(fminf(fmaxf(a_lx, a_hx), fmaxf(a_ly, a_hy)),
                                      fminf(fmaxf(a_lz, a_hz), h.t));
            const float tmin1 = fmaxf(fmaxf(fminf(b_lx, b_hx), fminf(b_ly, b_hy)),
                                      fmaxf(fminf(b_lz, b_hz), 0.0f));
            const float tmax1 = fminf(fminf(fmaxf(b_lx, b_hx), fmaxf(b_ly, b_hy)),
                                      fminf(fmaxf(b_lz, b_hz), h.t));
            const bool hit0 = tmin0 <= tmax0;
            const bool hit1 = tmin1 <= tmax1;
            if (hit0 && hit1) {
                const bool first0 = tmin0 <= tmin1;
                stack[sp * stride] = first0 ? cc.y : cc.x;
                ++sp;
                ref = first0 ? cc.x : cc.y;
            } else if (hit0) {
                ref = cc.x;
            } else if (hit1) {
                ref = cc.y;
            } else {
                if (sp == 0) break;
                --sp;
                ref = stack[sp * stride];
            }
        } else {
            const int32_t lr = ~ref;
            const int32_t first = lr >> 3;
            const int32_t cnt = (lr & 7) + 1;
            for (int i = 0; i < cnt; ++i) {
                if (COUNT) ++n_tris;
                const float4* tp = reinterpret_cast<const float4*>(sc.tris + first + i);
                const float4 t0 = tp[0];
                const float4 t1 = tp[1];
                const float4 t2 = tp[2];
                const V3 e1 = v3(t1.x, t1.y, t1.z);
                const V3 e2 = v3(t2.x, t2.y, t2.z);
                const V3 pv = cross(d, e2);
                const float det = dot(e1, pv);
                if (det == 0.0f) continue;
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
                    h.leaf = first + i;
                    best_orig = orig;
                }
            }
            if (sp == 0) break;
            --sp;
            ref = stack[sp * stride];
        }
    }
    return h;
}

// Radiance toward the ray origin at a hit: barycentric blend of the corner
// cache values plus the triangle's emission; zero on a miss.
__device__ __forceinline__ V3 radiance(const DeviceScene& sc, const Hit& h) {
    if (h.leaf < 0) return v3(0.0f, 0.0f, 0.0f);
    const float4* rp = reinterpret_cast<const float4*>(sc.rad + h.leaf);
    const float4 r0 = rp[0];
    const float4 r1 = rp[1];
    const float4 r2 = rp[2];
    const float w0 = 1.0f - h.u - h.v;
    return v3(w0 * r0.x + h.u * r0.w + h.v * r1.z + r2.y,
              w0 * r0.y + h.u * r1.x + h.v * r1.w + r2.z,
              w0 * r0.z + h.u * r1.y + h.v * r2.x + r2.w);
}

// Sum over the 64 lanes of a wave by a fixed xor butterfly: every lane ends
// with the same, order-fixed total.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace dev
}  // namespace fipt
