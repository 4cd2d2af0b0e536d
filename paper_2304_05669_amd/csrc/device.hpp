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
    // The key (wave-uniform in every caller) passes through an empty
    // statement, so the twenty round keys are formed here with scalar adds:
    // a loop-invariant seed otherwise has all of them hoisted out of the
    // sampling loop, and the bake, short of scalar registers, spills them
    // to vector lanes (a vector instruction per key on every refill).
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply gives both halves of a product
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
        const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
        // (three-way exclusive or in one instruction: truth table 0x96)
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// The even bits of x (bit 2i moved to bit i), packed into the low half.
__device__ __forceinline__ uint32_t even_bits(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// The uniforms (xi1, xi2) in [0, 1)^2 of sample s of a lobe's n samples,
// stratified along a curve over the unit square.  With the Philox block u
// of counter (p low, p high, lobe, s) and w = floor(2^32 / n) (0 standing
// for 2^32, n = 1), the position U = s w + floor(u0 w / 2^32) lies in the
// s-th of n equal segments of the 32-bit line.  U's top four bits number
// the cells of the 4 x 4 grid along a Hilbert curve (table: cell d is the
// nibble d of 0x3267BFEA9DC84510, column in its low two bits, row in the
// high two); the other 28 bits, read as a Morton code, place the point in
// that cell (14 bits per axis); the top bytes of u1 and u2 give the low 8
// bits of the two 24-bit results.  Samples with nearby indices get nearby
// directions (the Hilbert order has no jump across the square), and the
// estimate is stratified.  Both values are exact in float.
__device__ __forceinline__ void lobe_uniforms(uint64_t seed, int64_t p, int lobe, int s,
                                              uint32_t w, float& xi1, float& xi2) {
    const uint4 c = make_uint4((uint32_t)(uint64_t)p, (uint32_t)((uint64_t)p >> 32),
                               (uint32_t)lobe, (uint32_t)s);
    const uint4 u = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint32_t U = w == 0 ? u.x : (uint32_t)s * w + __umulhi(u.x, w);
    const uint32_t d = U >> 28;
    const uint32_t cell = ((d < 8 ? 0x9DC84510u : 0x3267BFEAu) >> ((d & 7u) * 4u)) & 15u;
    const uint32_t X = ((cell & 3u) << 14) | even_bits(U & 0x0FFFFFFFu);
    const uint32_t Y = ((cell >> 2) << 14) | even_bits((U >> 1) & 0x07FFFFFFu);
    xi1 = (float)((X << 8) | (u.y >> 24)) * (1.0f / 16777216.0f);
    xi2 = (float)((Y << 8) | (u.z >> 24)) * (1.0f / 16777216.0f);
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
// Reciprocal square root by the hardware instruction, for arguments known to
// be at least 1 (where rsqrtf gives the same instruction's result after a
// test for denormal inputs that cannot occur).
__device__ __forceinline__ float rsq_ge1(float x) { return __builtin_amdgcn_rsqf(x); }

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

// Hit distance of a ray that has hit nothing yet: the largest finite float,
// so that the +inf key of a missed child box always lies beyond it (the
// node step visits a child when its key is at most the hit distance).
constexpr float kNoHit = 3.40282347e+38f;

// Per-ray constants of the slab test against node bounds in units of
// `scale`: the inverse direction times the unit (a power of two, so the
// product is exact) and the origin times the inverse direction.
struct RaySlab {
    float ax, ay, az, oxi, oyi, ozi;
};
__device__ __forceinline__ RaySlab ray_slab(V3 o, V3 d, float scale) {
    const float dx = fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x);
    const float dy = fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y);
    const float dz = fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z);
    const float ix = __builtin_amdgcn_rcpf(dx);
    const float iy = __builtin_amdgcn_rcpf(dy);
    const float iz = __builtin_amdgcn_rcpf(dz);
    RaySlab r;
    r.ax = ix * scale;
    r.ay = iy * scale;
    r.az = iz * scale;
    r.oxi = o.x * ix;
    r.oyi = o.y * iy;
    r.ozi = o.z * iz;
    return r;
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

// The low / high half of a 32-bit word as a float (folded into the
// mixed-precision FMA that consumes it).
__device__ __forceinline__ float half_lo(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
}
__device__ __forceinline__ float half_hi(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// Slab test of one child box against [0, inf) from its near and far
// planes as half-precision offsets from the node origin: the distance to
// plane (org + off) 2^E is fma(off, a, org a - o ix) with a = ix 2^E.
// Returns the entry distance, or +inf when the box is missed.  An unused
// slot (low offsets +inf, high -inf) has near distance +inf and far
// distance -inf whatever the direction.  The current hit distance is not
// clipped in here: the caller compares the entry distance with it, once
// per child after the sort (the same boxes are visited, in the same order,
// as with the clipped interval, for one instruction less per child).
__device__ __forceinline__ float box_entry(float nx, float fx, float ny, float fy, float nz,
                                           float fz, float ax, float bx, float ay, float by,
                                           float az, float bz) {
    const float tn = fmaxf(fmaxf(fmaf(nx, ax, bx), fmaf(ny, ay, by)), fmaxf(fmaf(nz, az, bz), 0.0f));
    const float tf = fminf(fminf(fmaf(fx, ax, bx), fmaf(fy, ay, by)), fmaf(fz, az, bz));
    return tn <= tf ? tn : INFINITY;
}

// Pop the next entry of a lane's stack into `ref` (kDone when it is
// empty).  `top` is the lane's next free slot, `bottom` its first; slots
// are `stride` ints apart.
__device__ __forceinline__ void stack_pop(int32_t& ref, int32_t*& top, const int32_t* bottom,
                                          int stride) {
    if (top == bottom) {
        ref = kDone;
    } else {
        top -= stride;
        ref = *top;
    }
}

// One step of closest-hit traversal at 4-wide node `ref`: the children the
// ray enters no later than `tmax` (the current hit distance, finite) are
// visited nearest first; the nearest becomes `ref`, the others are pushed
// farthest first.  With no child hit, the next entry is popped
// (kDone when the stack is empty).  An inner reference is the node's byte
// offset (below 2^31: the builder rejects trees of more than kMaxNodes4
// nodes).
__device__ __forceinline__ void node4_step(const Bvh4Node* nodes, int32_t& ref, int32_t*& top,
                                           const int32_t* bottom, int stride, const RaySlab& r,
                                           float tmax) {
    const char* nb = reinterpret_cast<const char*>(nodes) + (uint32_t)ref;
    const int4 qx = load_global(reinterpret_cast<const int4*>(nb));
    const int4 qy = load_global(reinterpret_cast<const int4*>(nb + 16));
    const int4 qz = load_global(reinterpret_cast<const int4*>(nb + 32));
    const float4 og = load_global(reinterpret_cast<const float4*>(nb + 48));
    const int4 ch = load_global(reinterpret_cast<const int4*>(nb + 64));
    int32_t c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
    // keep the child load in the same batch as the box loads (otherwise it
    // is sunk below the miss branch and costs a second memory round trip)
    asm volatile("" : : "v"(c0), "v"(c1), "v"(c2), "v"(c3));
    // per axis: distance at the node origin
    const float ax = r.ax, ay = r.ay, az = r.az;
    const float bx = fmaf(og.x, ax, -r.oxi);
    const float by = fmaf(og.y, ay, -r.oyi);
    const float bz = fmaf(og.z, az, -r.ozi);
    // near planes are the low bounds for a positive direction component,
    // else the high bounds: words (lo0|lo1, lo2|lo3, hi0|hi1, hi2|hi3)
    const bool sx = ax < 0.0f, sy = ay < 0.0f, sz = az < 0.0f;
    const uint32_t nx01 = sx ? qx.z : qx.x, nx23 = sx ? qx.w : qx.y;
    const uint32_t fx01 = sx ? qx.x : qx.z, fx23 = sx ? qx.y : qx.w;
    const uint32_t ny01 = sy ? qy.z : qy.x, ny23 = sy ? qy.w : qy.y;
    const uint32_t fy01 = sy ? qy.x : qy.z, fy23 = sy ? qy.y : qy.w;
    const uint32_t nz01 = sz ? qz.z : qz.x, nz23 = sz ? qz.w : qz.y;
    const uint32_t fz01 = sz ? qz.x : qz.z, fz23 = sz ? qz.y : qz.w;
    float k0 = box_entry(half_lo(nx01), half_lo(fx01), half_lo(ny01), half_lo(fy01), half_lo(nz01),
                         half_lo(fz01), ax, bx, ay, by, az, bz);
    float k1 = box_entry(half_hi(nx01), half_hi(fx01), half_hi(ny01), half_hi(fy01), half_hi(nz01),
                         half_hi(fz01), ax, bx, ay, by, az, bz);
    float k2 = box_entry(half_lo(nx23), half_lo(fx23), half_lo(ny23), half_lo(fy23), half_lo(nz23),
                         half_lo(fz23), ax, bx, ay, by, az, bz);
    float k3 = box_entry(half_hi(nx23), half_hi(fx23), half_hi(ny23), half_hi(fy23), half_hi(nz23),
                         half_hi(fz23), ax, bx, ay, by, az, bz);
    // sorting network on four keys; a missed child keeps key +inf and one
    // entered beyond the current hit a key above tmax (finite: kNoHit
    // before the first hit), so both sort after every child to visit, and
    // the sorted keys compared with tmax say which children to visit
    order2(k0, c0, k1, c1);
    order2(k2, c2, k3, c3);
    order2(k0, c0, k2, c2);
    order2(k1, c1, k3, c3);
    order2(k1, c1, k2, c2);
    if (!(k0 <= tmax)) {
        stack_pop(ref, top, bottom, stride);
        return;
    }
    if (k3 <= tmax) {
        *top = c3;
        top += stride;
    }
    if (k2 <= tmax) {
        *top = c2;
        top += stride;
    }
    if (k1 <= tmax) {
        *top = c1;
        top += stride;
    }
    ref = c0;
}

// ---- the chain of boxes around a point ------------------------------------
// Every ray of a point starts at the same origin o, so every ray walks the
// same nodes first: while some child box of the current node contains o,
// that child is entered at distance 0, nearest of all, and only its
// siblings differ from ray to ray.  The bake finds that chain once per point
// and starts each ray below it, having tested only the siblings of the
// chain's children.  Which child is entered does not change the result: the
// chain's child is visited whether or not a given ray's slab test would
// accept it, and every sibling the ray's test accepts is pushed, so every
// box the plain traversal would visit is still visited.
constexpr int kChainMax = 16;   // levels kept (one per lane of the first 16)

// Node data through the constant address space: with a wave-uniform node
// the compiler reads it with scalar loads into scalar registers.
typedef const __attribute__((address_space(4))) int4* cint4p;
typedef const __attribute__((address_space(4))) float4* cfloat4p;
__device__ __forceinline__ int4 load_uniform(const void* p) {
    const gint4 v = *(const __attribute__((address_space(4))) gint4*)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 load_uniform_f(const void* p) {
    const gfloat4 v = *(const __attribute__((address_space(4))) gfloat4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Half j of the four packed in a (lo01, lo23) or (hi01, hi23) word pair.
template <int J>
__device__ __forceinline__ float half_of(uint32_t w01, uint32_t w23) {
    return J == 0 ? half_lo(w01) : J == 1 ? half_hi(w01) : J == 2 ? half_lo(w23) : half_hi(w23);
}

// The chain of point origin o (same value in every lane): lane i of `chain`
// receives node | slot for level i (the node's byte offset, whose low seven
// bits are zero, and which of its children contains o); returns the number
// of levels; `end` is the reference the
// traversal continues from (the last chain child, or the node where no
// child contains o, or the root).  Containment is tested on the decoded
// half-precision bounds in units of the node scale.
__device__ __forceinline__ int point_chain(const Bvh4Node* nodes, float scale, V3 o, int lane,
                                           int32_t& chain, int32_t& end) {
    const float inv = 1.0f / scale;   // a power of two: exact
    const float ux = o.x * inv, uy = o.y * inv, uz = o.z * inv;
    int L = 0;
    int32_t node = 0;
    chain = 0;
    while (L < kChainMax) {
        const char* nb = reinterpret_cast<const char*>(nodes) + (uint32_t)node;
        const int4 qx = load_uniform(nb), qy = load_uniform(nb + 16), qz = load_uniform(nb + 32);
        const float4 og = load_uniform_f(nb + 48);
        const int4 ch = load_uniform(nb + 64);
        int slot = -1;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const uint32_t lx = j < 2 ? qx.x : qx.y, hx = j < 2 ? qx.z : qx.w;
            const uint32_t ly = j < 2 ? qy.x : qy.y, hy = j < 2 ? qy.z : qy.w;
            const uint32_t lz = j < 2 ? qz.x : qz.y, hz = j < 2 ? qz.z : qz.w;
            const float x0 = og.x + ((j & 1) ? half_hi(lx) : half_lo(lx));
            const float x1 = og.x + ((j & 1) ? half_hi(hx) : half_lo(hx));
            const float y0 = og.y + ((j & 1) ? half_hi(ly) : half_lo(ly));
            const float y1 = og.y + ((j & 1) ? half_hi(hy) : half_lo(hy));
            const float z0 = og.z + ((j & 1) ? half_hi(lz) : half_lo(lz));
            const float z1 = og.z + ((j & 1) ? half_hi(hz) : half_lo(hz));
            const bool in = (x0 <= ux) & (ux <= x1) & (y0 <= uy) & (uy <= y1) & (z0 <= uz) &
                            (uz <= z1);
            slot = in ? j : slot;   // the lowest slot that contains o
        }
        slot = __builtin_amdgcn_readfirstlane(slot);
        if (slot < 0) break;
        if (lane == L) chain = (int32_t)((uint32_t)node | (uint32_t)slot);
        ++L;
        const int32_t child = __builtin_amdgcn_readfirstlane(
            slot == 0 ? ch.x : slot == 1 ? ch.y : slot == 2 ? ch.z : ch.w);
        if (child < 0) {
            end = child;   // a leaf (an unused slot never contains o)
            return L;
        }
        node = child;
    }
    end = node;
    return L;
}

// Entry distance of child J of a node whose planes the lane does not
// select beforehand (the node's words are wave-uniform): both plane
// distances per axis, then near and far by the direction's sign.  No hit
// yet, so the far bound is not clipped.
template <int J>
__device__ __forceinline__ float chain_key(const int4& qx, const int4& qy, const int4& qz,
                                           const RaySlab& r, float bx, float by, float bz) {
    const float lx = fmaf(half_of<J>(qx.x, qx.y), r.ax, bx), hx = fmaf(half_of<J>(qx.z, qx.w), r.ax, bx);
    const float ly = fmaf(half_of<J>(qy.x, qy.y), r.ay, by), hy = fmaf(half_of<J>(qy.z, qy.w), r.ay, by);
    const float lz = fmaf(half_of<J>(qz.x, qz.y), r.az, bz), hz = fmaf(half_of<J>(qz.z, qz.w), r.az, bz);
    const bool sx = r.ax < 0.0f, sy = r.ay < 0.0f, sz = r.az < 0.0f;
    const float tn = fmaxf(fmaxf(sx ? hx : lx, sy ? hy : ly), fmaxf(sz ? hz : lz, 0.0f));
    const float tf = fminf(fminf(sx ? lx : hx, sy ? ly : hy), sz ? lz : hz);
    return tn <= tf ? tn : INFINITY;
}

template <int A, int B, int C>
__device__ __forceinline__ void chain_siblings3(const int4& qx, const int4& qy, const int4& qz,
                                                const int4& ch, const RaySlab& r, float bx,
                                                float by, float bz, int32_t*& top, int stride) {
    float ka = chain_key<A>(qx, qy, qz, r, bx, by, bz);
    float kb = chain_key<B>(qx, qy, qz, r, bx, by, bz);
    float kc = chain_key<C>(qx, qy, qz, r, bx, by, bz);
    const int32_t refs[4] = {ch.x, ch.y, ch.z, ch.w};
    int32_t ca = refs[A], cb = refs[B], cc = refs[C];
    order2(ka, ca, kb, cb);
    order2(kb, cb, kc, cc);
    order2(ka, ca, kb, cb);
    if (kc < INFINITY) {
        *top = cc;
        top += stride;
    }
    if (kb < INFINITY) {
        *top = cb;
        top += stride;
    }
    if (ka < INFINITY) {
        *top = ca;
        top += stride;
    }
}

// One chain level for a ray: the three siblings of the chain's child at
// node `node` (a byte offset; slot `skip`) are tested and the hit ones pushed, farthest
// first, as the plain step would push them (the chain's child, entered at
// distance 0, is visited next without a push).
__device__ __forceinline__ void chain_step(const Bvh4Node* nodes, int32_t node, int skip,
                                           const RaySlab& r, int32_t*& top, int stride) {
    const char* nb = reinterpret_cast<const char*>(nodes) + (uint32_t)node;
    const int4 qx = load_uniform(nb), qy = load_uniform(nb + 16), qz = load_uniform(nb + 32);
    const float4 og = load_uniform_f(nb + 48);
    const int4 ch = load_uniform(nb + 64);
    const float bx = fmaf(og.x, r.ax, -r.oxi);
    const float by = fmaf(og.y, r.ay, -r.oyi);
    const float bz = fmaf(og.z, r.az, -r.ozi);
    switch (skip) {
        case 0: chain_siblings3<1, 2, 3>(qx, qy, qz, ch, r, bx, by, bz, top, stride); break;
        case 1: chain_siblings3<0, 2, 3>(qx, qy, qz, ch, r, bx, by, bz, top, stride); break;
        case 2: chain_siblings3<0, 1, 3>(qx, qy, qz, ch, r, bx, by, bz, top, stride); break;
        default: chain_siblings3<0, 1, 2>(qx, qy, qz, ch, r, bx, by, bz, top, stride); break;
    }
}

// Triangle test (Moller-Trumbore) of leaf-order triangle `i`; updates the
// closest hit, exact distance ties going to the lower original index.  A
// triangle parallel to the ray (det = 0) needs no early exit: its
// reciprocal is infinite, so u, v and t are infinite or NaN and the inside
// test fails; without the branch all three loads issue together (the
// branch let the compiler delay the vertex load behind it, a second memory
// round trip per test).
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
    const RaySlab r = ray_slab(o, d, sc.box_scale);
    Hit h;
    h.leaf = -1;
    h.t = kNoHit;
    h.u = h.v = 0.0f;
    int32_t best_orig = INT_MAX;
    int32_t ref = 0;
    int32_t* top = stack;
    while (ref != kDone) {
        if (ref >= 0) {
            if (COUNT) ++n_nodes;
            node4_step(sc.nodes, ref, top, stack, stride, r, h.t);
        } else {
            const int32_t lr = ~ref;
            const int32_t first = lr >> 3;
            const int32_t cnt = (lr & 7) + 1;
            for (int i = 0; i < cnt; ++i) {
                if (COUNT) ++n_tris;
                tri_test(sc.tris, first + i, o, d, h, best_orig);
            }
            stack_pop(ref, top, stack, stride);
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

// Radiance at a hit with the voxel cache of Sec. 4.2: the value of the voxel
// that contains the hit point o + t d (nearest-voxel query), plus the
// triangle's emission (the last 16 bytes of its radiance record).  The
// voxel coordinate is clamped in float before the conversion, so points
// outside the grid read its border voxels and the conversion is exact.  The
// grid is sparse, in bricks of 4 x 4 x 4 voxels: the brick's occupancy word
// (bit mask of its 64 voxels and the count of occupied voxels in earlier
// bricks) locates the value, and empty voxels read zero without a second
// load.  Hits near each other on a surface fall in the same or adjacent
// bricks, so their words and values share cache lines.
__device__ __forceinline__ V3 radiance_voxel(const DeviceScene& sc, const Hit& h, const V3& o,
                                             const V3& d) {
    if (h.leaf < 0) return v3(0.0f, 0.0f, 0.0f);
    const float4 e = load_global(reinterpret_cast<const float4*>(sc.rad + h.leaf) + 2);
    const float top = (float)(sc.vox_res - 1);
    const float ux = fminf(fmaxf((fmaf(h.t, d.x, o.x) - sc.vox_lo[0]) * sc.vox_scale[0], 0.0f), top);
    const float uy = fminf(fmaxf((fmaf(h.t, d.y, o.y) - sc.vox_lo[1]) * sc.vox_scale[1], 0.0f), top);
    const float uz = fminf(fmaxf((fmaf(h.t, d.z, o.z) - sc.vox_lo[2]) * sc.vox_scale[2], 0.0f), top);
    // brick of 4 x 4 x 4 voxels and the voxel's bit in it (res <= 512, so
    // 32-bit indices)
    const uint32_t ix = (uint32_t)ux, iy = (uint32_t)uy, iz = (uint32_t)uz;
    const uint32_t nb = (uint32_t)sc.vox_bricks;
    const uint32_t brick = ((iz >> 2) * nb + (iy >> 2)) * nb + (ix >> 2);
    const int4 w = load_global(reinterpret_cast<const int4*>(sc.vox_words) + brick);
    const uint64_t m = ((uint64_t)(uint32_t)w.y << 32) | (uint32_t)w.x;
    const int b = (int)((((iz & 3u) << 2 | (iy & 3u)) << 2) | (ix & 3u));
    V3 c = v3(e.y, e.z, e.w);
    if ((m >> b) & 1ull) {
        const uint32_t idx = (uint32_t)w.z + (uint32_t)__popcll(m & ((1ull << b) - 1ull));
        const float4 q = load_global(sc.vox + idx);
        c = v3(c.x + q.x, c.y + q.y, c.z + q.z);
    }
    return c;
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

// ---- work distribution shared by the persistent bake kernels ---------------
// Lobe of flattened sample q: 0 for the first spp_d (diffuse) samples, then
// 1 + (q - spp_d) / spp_s.  The quotient is below 17 and r < 2^20 (spp <=
// 65536, K <= 16), so the float estimate is off by at most one, at exact
// multiples, and the correction makes it exact.
__device__ __forceinline__ int lobe_of(int q, int spp_d, int spp_s) {
    if (q < spp_d) return 0;
    const int r = q - spp_d;
    int l = (int)((float)r * __builtin_amdgcn_rcpf((float)spp_s));
    if ((int)__umul24((unsigned)l, (unsigned)spp_s) > r) --l;
    else if ((int)__umul24((unsigned)(l + 1), (unsigned)spp_s) <= r) ++l;
    return 1 + l;
}

// Output plane of accumulator slot j: slot 0..2 -> Ld; slot 3 + 6k + c ->
// Ls0 level k; slot 3 + 6k + 3 + c -> Ls1 level k.
__device__ __forceinline__ int slot_plane(int j, int K) {
    if (j < 3) return j;
    const int r = j - 3, k = r / 6, c = r - 6 * k;
    return c < 3 ? 3 + 3 * k + c : 3 + 3 * K + 3 * k + (c - 3);
}


// The point index is the same in every lane of a wavefront; saying so lets
// the compiler keep the point's data in scalar registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Dynamic point hand-out.  The points of a launch are cut into kXcdCount
// contiguous shares, one per XCD, each with its own counter: a wavefront
// takes the next point of its XCD's share, so each XCD's L2 sees one
// contiguous run of points; when that share is used up it takes points from
// the other shares in turn.  Returns -1 once every share is exhausted
// (`tried` counts the shares found empty).  Each point's result does not
// depend on which wavefront bakes it.
__device__ __forceinline__ int64_t next_point(int32_t* counters, int home, int& tried,
                                              int64_t total, int lane) {
    while (tried < kXcdCount) {
        const int x = (home + tried) % kXcdCount;
        int32_t grab = 0;
        if (lane == 0) grab = atomicAdd(counters + x, 1);
        const int64_t p = total * x / kXcdCount + __builtin_amdgcn_readfirstlane(grab);
        if (p < total * (x + 1) / kXcdCount) return p;
        ++tried;
    }
    return -1;
}

}  // namespace dev
}  // namespace fipt
