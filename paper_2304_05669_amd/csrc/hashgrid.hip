// The paper's material network for gfx950 (Eq. 14; architecture from its
// network paragraph): (a, sigma, m) = Sigmoid(MLP(hash encoding of x)), with
// a multiresolution hash encoding of 32 levels x 2^19 entries x 2 features
// (base resolution 16, scale 2 per level: level l has 16 * 2^l cells per
// axis over the scene box; levels whose vertices fit the table are indexed
// densely, the others by the spatial hash with the primes 1, 2654435761,
// 805459861) and an MLP of two hidden layers of 64 (ReLU, no biases).
//
// Parameters, one float array: tables [32][2^19][2], then W1 [64][64],
// W2 [64][64], W3 [5][64] (row = output).
//
// Forward: one lane per point for the encoding (the 256 table gathers per
// point, 8 vertices x 32 levels of 8 bytes, are the memory traffic; the
// tables, 134 MB, live in HBM and the MALL) and the two hidden layers on the
// matrix cores over the wavefront's 64 points (see below), the weights in
// LDS; the five outputs on the vector ALUs.
//
// Backward: each wavefront recomputes the forward pass of its 64 points,
// back-propagates through the MLP (W2^T and W1^T on the matrix cores too),
// stores the per-level feature gradients (W1^T d1, two per level) and the
// activations and layer gradients in a workspace.  The table
// gradient is then a gather: a plan built once for the point set lists, per
// level, every (point, corner) with a nonzero trilinear weight sorted by
// table slot (then point, then corner), and one group of lanes per slot sums
// weight x feature gradient over its list in that order, in double, adding
// the total into the slot's entry; no atomics, so the table gradient is
// reproducible bit for bit.  The weight gradients are sums over points of
// outer products (three small GEMMs with the point count as the reduction
// dimension): a split-K kernel forms one 64 x 64 partial per chunk of 2048
// points on the matrix cores, and a final kernel adds the partials in chunk
// order, so weight gradients are reproducible too.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fipt_internal.hpp"

namespace fipt {
namespace {

constexpr int kLevels = FIPT_HG_LEVELS;
constexpr int kFeat = 2;
constexpr uint32_t kT = 1u << FIPT_HG_LOG2_TABLE;
constexpr int kIn = kLevels * kFeat;   // 64
constexpr int kHid = 64;
constexpr int kOut = 5;
constexpr int64_t kTable = (int64_t)kLevels * kT * kFeat;
constexpr int kW1 = kHid * kIn, kW2 = kHid * kHid, kW3 = kOut * kHid;
constexpr int kWeights = kW1 + kW2 + kW3;   // 8512
constexpr int kBlock = 256;
constexpr int kChunk = 2048;              // points per weight-gradient partial
constexpr int kWsRows = 3 * 64 + 2 * 64 + kOut;   // e, h1, h2, d1, d2, d3
constexpr int kFeatGradRows = kLevels * kFeat;     // per-level feature gradients, [32][n] float2

struct HgArgs {
    const float* params;
    const float* pos;
    int64_t ps;
    int64_t n;
    float lo[3];
    float inv[3];
};

// Cell of coordinate p in [0, 1] at a level of N cells: lower vertex (low 32
// bits of the integer coordinate) and fraction, exact in single precision.
__device__ __forceinline__ void cell(float p, float nl, uint32_t& c, float& f) {
    const float u = p * nl;
    const float cf = fminf(floorf(u), nl - 1.0f);
    f = u - cf;
    c = (uint32_t)(uint64_t)cf;
}

// Table slots and trilinear weights of the 8 vertices of the point's cell at
// level l (corner bit 0/1/2 = +1 along x/y/z).  The level is a run-time
// value so that no register array is indexed by it.
__device__ __forceinline__ void corners(int l, const float p[3], uint32_t idx[8], float w[8]) {
    const float nl = 16.0f * (float)(1u << l);   // exact power of two
    uint32_t cx, cy, cz;
    float fx, fy, fz;
    cell(p[0], nl, cx, fx);
    cell(p[1], nl, cy, fy);
    cell(p[2], nl, cz, fz);
    const bool dense = l < 3;   // (16 * 2^l + 1)^3 <= 2^19
    const uint32_t r = (16u << (l & 3)) + 1u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        w[k] = (dx ? fx : 1.0f - fx) * (dy ? fy : 1.0f - fy) * (dz ? fz : 1.0f - fz);
        const uint32_t x = cx + dx, y = cy + dy, z = cz + dz;
        idx[k] = dense ? x + y * r + z * r * r
                       : (x ^ (y * 2654435761u) ^ (z * 805459861u)) & (kT - 1u);
    }
}

// Unit-cube position of point i (single precision, as specified).
__device__ __forceinline__ void unit_pos(const HgArgs& a, int64_t i, float p[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
        p[k] = fminf(fmaxf((a.pos[k * a.ps + i] - a.lo[k]) * a.inv[k], 0.0f), 1.0f);
}

// ---- the backward pass on the matrix cores -----------------------------------
// One wavefront holds 64 points as two tiles of 32 (points 0-31 and 32-63 of
// the wavefront).  A 64 x 64 layer over them is four 32 x 32 output tiles of
// v_mfma_f32_32x32x2f32, two input features per instruction: lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32], and accumulator register r of lane
// l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] (dfeat below).  The
// encoding arrives one level (two features) at a time with a lane per point;
// v_permlane32_swap turns the two feature registers into the B operands of
// both point tiles.  A layer's output feeds the next layer as B without any
// data movement: its reduction takes the features in the order the output
// registers hold them (register r of the two half-waves, features f and
// f + 4), and the weights are read from LDS in that same order.  The weights
// live in LDS with rows of 65 floats, so that a row-wise read (W) and a
// column-wise read (W^T) both reach distinct banks across the 32 lanes.
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int kWs = 65;                                      // LDS row stride of W1 and W2
constexpr int kLdsW = 2 * kHid * kWs + kW3;                  // floats of weights in LDS

__device__ __forceinline__ int dfeat(int i, int r, int h) { return 32 * i + 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ v16f mfma2(float a, float b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// (lanes 0-31 of x, lanes 0-31 of y) and (lanes 32-63 of x, lanes 32-63 of y)
__device__ __forceinline__ void swap_halves(float x, float y, float& lo_pair, float& hi_pair) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    lo_pair = __uint_as_float(r[0]);
    hi_pair = __uint_as_float(r[1]);
}

// SAVED: the workspace already holds the encoding (rows 0-63, written by
// the forward pass of the same parameters and points), which is read
// instead of gathered from the tables again.
template <bool SAVED>
__global__ __launch_bounds__(kBlock) void k_hg_backward(HgArgs a, const float* __restrict__ gy,
                                                             int64_t gs, float* __restrict__ ws,
                                                             int64_t wn, float2* __restrict__ fgrad) {
    __shared__ float w[kLdsW];
    {
        const float* src = a.params + kTable;
        for (int q = threadIdx.x; q < kW1 + kW2; q += kBlock) {
            const int m = q / kW1, rc = q % kW1;
            w[m * kHid * kWs + (rc / kIn) * kWs + rc % kIn] = src[q];
        }
        for (int q = threadIdx.x; q < kW3; q += kBlock) w[2 * kHid * kWs + q] = src[kW1 + kW2 + q];
    }
    __syncthreads();
    const float* W1 = w;                   // W1[o][c] at o * kWs + c
    const float* W2 = w + kHid * kWs;      // W2[o][c] at o * kWs + c
    const float* W3 = w + 2 * kHid * kWs;  // W3[o][c] at o * 64 + c
    const int lane = threadIdx.x & 63, h = lane >> 5, lo = lane & 31;
    const int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63);
    const int64_t i = base + lane;          // this lane's point in the encoding
    const bool live = i < a.n;
    v16f z[2][2];                           // z1, then h1 = relu(z1): [output tile][point tile]
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) z[u][j][r] = 0.0f;
    {
        float p[3] = {0.0f, 0.0f, 0.0f};
        if (!SAVED && live) unit_pos(a, i, p);
        const float2* t2 = reinterpret_cast<const float2*>(a.params);
#pragma unroll 1
        for (int l = 0; l < kLevels; ++l) {
            float e0 = 0.0f, e1 = 0.0f;
            if (SAVED) {
                if (live) {
                    e0 = ws[(int64_t)(2 * l) * wn + i];
                    e1 = ws[(int64_t)(2 * l + 1) * wn + i];
                }
            } else {
                uint32_t idx[8];
                float wt[8];
                corners(l, p, idx, wt);
                const float2* t = t2 + (int64_t)l * kT;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (wt[k] != 0.0f) {
                        const float2 v = t[idx[k]];
                        e0 = fmaf(wt[k], v.x, e0);
                        e1 = fmaf(wt[k], v.y, e1);
                    }
                }
                if (live) {
                    ws[(int64_t)(2 * l) * wn + i] = e0;
                    ws[(int64_t)(2 * l + 1) * wn + i] = e1;
                }
            }
            float b0, b1;   // features 2l (lanes 0-31) and 2l + 1 (lanes 32-63) of point tiles 0 and 1
            swap_halves(e0, e1, b0, b1);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W1[(32 * u + lo) * kWs + 2 * l + h];
                z[u][0] = mfma2(av, b0, z[u][0]);
                z[u][1] = mfma2(av, b1, z[u][1]);
            }
        }
    }
    // h1 = relu(z1), stored (rows 64 + f)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                z[u][j][r] = fmaxf(z[u][j][r], 0.0f);
                const int64_t pt = base + 32 * j + lo;
                if (pt < a.n) ws[(int64_t)(64 + dfeat(u, r, h)) * wn + pt] = z[u][j][r];
            }
    // z2 = W2 h1, h2 = relu(z2), stored (rows 128 + f)
    v16f y[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) y[u][j][r] = 0.0f;
#pragma unroll
    for (int ui = 0; ui < 2; ++ui)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = dfeat(ui, r, h);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W2[(32 * u + lo) * kWs + c];
                y[u][0] = mfma2(av, z[ui][0][r], y[u][0]);
                y[u][1] = mfma2(av, z[ui][1][r], y[u][1]);
            }
        }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                y[u][j][r] = fmaxf(y[u][j][r], 0.0f);
                const int64_t pt = base + 32 * j + lo;
                if (pt < a.n) ws[(int64_t)(128 + dfeat(u, r, h)) * wn + pt] = y[u][j][r];
            }
    // outputs: each lane sums its half of the features of its two points;
    // the halves meet with a swap, one point per lane
    float d3[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float wv = W3[o * kHid + dfeat(u, r, h)];
                s0 = fmaf(wv, y[u][0][r], s0);
                s1 = fmaf(wv, y[u][1][r], s1);
            }
        float pa, pb;
        swap_halves(s0, s1, pa, pb);
        const float sv = pa + pb;           // point base + lane
        const float yv = 1.0f / (1.0f + expf(-sv));
        d3[o] = live ? gy[o * gs + i] * yv * (1.0f - yv) : 0.0f;
        if (live) ws[(int64_t)(320 + o) * wn + i] = d3[o];
    }
    // d2 = (W3^T d3) masked by h2 > 0, in y's registers (rows 256 + f); the
    // d3 of both point tiles reach every lane with a swap
    float da[kOut], db[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) swap_halves(d3[o], d3[o], da[o], db[o]);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = dfeat(u, r, h);
            float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
            for (int o = 0; o < kOut; ++o) {
                const float wv = W3[o * kHid + c];
                s0 = fmaf(wv, da[o], s0);
                s1 = fmaf(wv, db[o], s1);
            }
            y[u][0][r] = y[u][0][r] > 0.0f ? s0 : 0.0f;
            y[u][1][r] = y[u][1][r] > 0.0f ? s1 : 0.0f;
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                const int64_t pt = base + 32 * jj + lo;
                if (pt < a.n) ws[(int64_t)(256 + c) * wn + pt] = y[u][jj][r];
            }
        }
    // d1 = (W2^T d2) masked by h1 > 0, into z's registers (rows 192 + f)
    v16f g[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int r = 0; r < 16; ++r) g[u][jj][r] = 0.0f;
#pragma unroll
    for (int ui = 0; ui < 2; ++ui)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = dfeat(ui, r, h);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W2[c * kWs + 32 * u + lo];
                g[u][0] = mfma2(av, y[ui][0][r], g[u][0]);
                g[u][1] = mfma2(av, y[ui][1][r], g[u][1]);
            }
        }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                z[u][jj][r] = z[u][jj][r] > 0.0f ? g[u][jj][r] : 0.0f;
                const int64_t pt = base + 32 * jj + lo;
                if (pt < a.n) ws[(int64_t)(192 + dfeat(u, r, h)) * wn + pt] = z[u][jj][r];
            }
    // feature gradients W1^T d1: features 2l and 2l + 1 sit in registers r,
    // r + 1 (r even) of one lane, stored as one float2 per level
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int r = 0; r < 16; ++r) g[u][jj][r] = 0.0f;
#pragma unroll
    for (int ui = 0; ui < 2; ++ui)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = dfeat(ui, r, h);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W1[c * kWs + 32 * u + lo];
                g[u][0] = mfma2(av, z[ui][0][r], g[u][0]);
                g[u][1] = mfma2(av, z[ui][1][r], g[u][1]);
            }
        }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int64_t pt = base + 32 * jj + lo;
            if (pt < a.n) {
#pragma unroll
                for (int r = 0; r < 16; r += 2)
                    fgrad[(int64_t)(dfeat(u, r, h) >> 1) * wn + pt] = make_float2(g[u][jj][r], g[u][jj][r + 1]);
            }
        }
}

// The forward pass in the same layout: the two hidden layers on the matrix
// cores, the five outputs summed per half-wave on the vector ALUs.
// SAVE: the encoding also goes to rows 0-63 of the backward pass's
// workspace ws[.][wn], so that the backward pass need not gather it again.
template <bool SAVE>
__global__ __launch_bounds__(kBlock) void k_hg_forward(HgArgs a, float* __restrict__ out, int64_t os,
                                                       float* __restrict__ ws, int64_t wn) {
    __shared__ float w[kLdsW];
    {
        const float* src = a.params + kTable;
        for (int q = threadIdx.x; q < kW1 + kW2; q += kBlock) {
            const int m = q / kW1, rc = q % kW1;
            w[m * kHid * kWs + (rc / kIn) * kWs + rc % kIn] = src[q];
        }
        for (int q = threadIdx.x; q < kW3; q += kBlock) w[2 * kHid * kWs + q] = src[kW1 + kW2 + q];
    }
    __syncthreads();
    const float* W1 = w;
    const float* W2 = w + kHid * kWs;
    const float* W3 = w + 2 * kHid * kWs;
    const int lane = threadIdx.x & 63, h = lane >> 5, lo = lane & 31;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < a.n;
    v16f z[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) z[u][j][r] = 0.0f;
    {
        float p[3] = {0.0f, 0.0f, 0.0f};
        if (live) unit_pos(a, i, p);
        const float2* t2 = reinterpret_cast<const float2*>(a.params);
#pragma unroll 1
        for (int l = 0; l < kLevels; ++l) {
            uint32_t idx[8];
            float wt[8];
            corners(l, p, idx, wt);
            const float2* t = t2 + (int64_t)l * kT;
            float e0 = 0.0f, e1 = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (wt[k] != 0.0f) {
                    const float2 v = t[idx[k]];
                    e0 = fmaf(wt[k], v.x, e0);
                    e1 = fmaf(wt[k], v.y, e1);
                }
            }
            if (SAVE && live) {
                ws[(int64_t)(2 * l) * wn + i] = e0;
                ws[(int64_t)(2 * l + 1) * wn + i] = e1;
            }
            float b0, b1;
            swap_halves(e0, e1, b0, b1);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W1[(32 * u + lo) * kWs + 2 * l + h];
                z[u][0] = mfma2(av, b0, z[u][0]);
                z[u][1] = mfma2(av, b1, z[u][1]);
            }
        }
    }
    v16f y[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) y[u][j][r] = 0.0f;
#pragma unroll
    for (int ui = 0; ui < 2; ++ui)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = dfeat(ui, r, h);
            const float h0 = fmaxf(z[ui][0][r], 0.0f), h1 = fmaxf(z[ui][1][r], 0.0f);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float av = W2[(32 * u + lo) * kWs + c];
                y[u][0] = mfma2(av, h0, y[u][0]);
                y[u][1] = mfma2(av, h1, y[u][1]);
            }
        }
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float wv = W3[o * kHid + dfeat(u, r, h)];
                s0 = fmaf(wv, fmaxf(y[u][0][r], 0.0f), s0);
                s1 = fmaf(wv, fmaxf(y[u][1][r], 0.0f), s1);
            }
        float pa, pb;
        swap_halves(s0, s1, pa, pb);
        if (live) out[o * os + i] = 1.0f / (1.0f + expf(-(pa + pb)));
    }
}

// ---- table-gradient plan ---------------------------------------------------
// Sort keys of level l: the slot of each (point, corner) with a nonzero
// weight, kT (after every slot) for the others; values p << 3 | corner, in
// point order, so the stable radix sort leaves each slot's list in (point,
// corner) order.  `nnz` counts the nonzero weights.
__global__ __launch_bounds__(kBlock) void k_hgp_keys(HgArgs a, int l, uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals,
                                                     unsigned long long* __restrict__ nnz) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int c = 0;
    if (i < a.n) {
        float p[3];
        unit_pos(a, i, p);
        uint32_t idx[8];
        float w[8];
        corners(l, p, idx, w);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            keys[8 * i + k] = w[k] != 0.0f ? idx[k] : kT;
            vals[8 * i + k] = (uint32_t)(i << 3) | (uint32_t)k;
            c += w[k] != 0.0f;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nnz, (unsigned long long)c);
}

// Entries (p << 3 | corner, weight bits) of the sorted nonzero list.
__global__ __launch_bounds__(kBlock) void k_hgp_entries(HgArgs a, int l, const uint32_t* __restrict__ vals,
                                                        int64_t nnz, int2* __restrict__ ent) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nnz) return;
    const uint32_t e = vals[i];
    float p[3];
    unit_pos(a, e >> 3, p);
    uint32_t idx[8];
    float w[8];
    corners(l, p, idx, w);
    float wk = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) wk = (int)(e & 7) == k ? w[k] : wk;
    ent[i] = make_int2((int)e, __float_as_int(wk));
}

// Slot ranges: off[s] = the first sorted entry whose slot is >= s (a binary
// search per slot), so off[kT] = nnz.
__global__ __launch_bounds__(kBlock) void k_hgp_offsets(const uint32_t* __restrict__ keys, int64_t nnz,
                                                        uint32_t* __restrict__ off) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > (int64_t)kT) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < s) lo = mid + 1;
        else hi = mid;
    }
    off[s] = (uint32_t)lo;
}

// Table gradient of one level, slots of at most kHeavy entries: L lanes per
// slot (a power of two up to 64); lane j sums entries j, j + L, ... of the
// slot's list in double (four entries' loads, then their four gradient
// loads, in flight together), a fixed butterfly adds the L partial sums, and
// the first lane adds the total into the slot's two features.
constexpr uint32_t kHeavy = 256;

__device__ __forceinline__ void gather_sum(const int2* __restrict__ ent, const float2* __restrict__ fg,
                                           uint32_t first, uint32_t e1, uint32_t stride, double& s0,
                                           double& s1) {
    for (uint32_t e = first; e < e1; e += 4 * stride) {
        int2 en[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) en[u] = ent[min(e + u * stride, e1 - 1)];
        float2 d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = fg[(uint32_t)en[u].x >> 3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (e + u * stride < e1) {
                const double w = (double)__int_as_float(en[u].y);
                s0 += w * (double)d[u].x;
                s1 += w * (double)d[u].y;
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_hg_table_grad(const int2* __restrict__ ent,
                                                          const uint32_t* __restrict__ off,
                                                          const float2* __restrict__ fg, int64_t n_slots,
                                                          int L, float* __restrict__ t) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t slot = g / L;
    const int j = (int)(g % L);
    double s0 = 0.0, s1 = 0.0;
    uint32_t e0 = 0, e1 = 0;
    if (slot < n_slots) {
        e0 = off[slot];
        e1 = off[slot + 1];
        if (e1 - e0 > kHeavy) e1 = e0;   // a heavy slot: k_hg_table_grad_heavy
        gather_sum(ent, fg, e0 + j, e1, L, s0, s1);
    }
    for (int m = 1; m < L; m <<= 1) {
        s0 += __shfl_xor(s0, m, 64);
        s1 += __shfl_xor(s1, m, 64);
    }
    if (j == 0 && e1 > e0) {
        t[2 * slot] += (float)s0;
        t[2 * slot + 1] += (float)s1;
    }
}

// The heavy slots of a level (more than kHeavy entries; the plan lists
// them): one workgroup per slot, thread j summing entries j, j + kBlock, ...;
// each wavefront's butterfly, then the four wavefront totals in order.
__global__ __launch_bounds__(kBlock) void k_hg_table_grad_heavy(const int2* __restrict__ ent,
                                                                const uint32_t* __restrict__ off,
                                                                const uint32_t* __restrict__ heavy,
                                                                const float2* __restrict__ fg,
                                                                float* __restrict__ t) {
    __shared__ double part[kBlock / 64][2];
    const uint32_t slot = heavy[blockIdx.x];
    const uint32_t e0 = off[slot], e1 = off[slot + 1];
    double s0 = 0.0, s1 = 0.0;
    gather_sum(ent, fg, e0 + threadIdx.x, e1, kBlock, s0, s1);
    for (int m = 1; m < 64; m <<= 1) {
        s0 += __shfl_xor(s0, m, 64);
        s1 += __shfl_xor(s1, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6][0] = s0;
        part[threadIdx.x >> 6][1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            a += part[w][0];
            b += part[w][1];
        }
        t[2 * slot] += (float)a;
        t[2 * slot + 1] += (float)b;
    }
}

// Staging pieces of k_hg_wgrad<true>: thread t's piece j of a 64-point tile
// is row (t + 256 j) / 16, points 4 ((t + 256 j) % 16) .. + 3 of the A
// operand (rows of A past `rows` are zero) and of the B operand.
__device__ __forceinline__ void wgrad_piece(const float* __restrict__ ws, int64_t wn, int64_t p0,
                                            int64_t p_end, int idx, int rows, int a_row0, int b_row0,
                                            float4& ra, float4& rb) {
    const int r = idx >> 4, c = (idx & 15) * 4;
    const int64_t pp = p0 + c;
    const float* pa = ws + (int64_t)(a_row0 + r) * wn;
    const float* pb = ws + (int64_t)(b_row0 + r) * wn;
    if (pp + 3 < p_end) {
        ra = r < rows ? *reinterpret_cast<const float4*>(pa + pp) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        rb = *reinterpret_cast<const float4*>(pb + pp);
    } else {
        ra = make_float4(r < rows && pp < p_end ? pa[pp] : 0.0f, r < rows && pp + 1 < p_end ? pa[pp + 1] : 0.0f,
                         r < rows && pp + 2 < p_end ? pa[pp + 2] : 0.0f, 0.0f);
        rb = make_float4(pp < p_end ? pb[pp] : 0.0f, pp + 1 < p_end ? pb[pp + 1] : 0.0f,
                         pp + 2 < p_end ? pb[pp + 2] : 0.0f, 0.0f);
    }
}
__device__ __forceinline__ void wgrad_fetch(const float* __restrict__ ws, int64_t wn, int64_t p0,
                                            int64_t p_end, int t, int rows, int a_row0, int b_row0,
                                            float4& ra0, float4& rb0, float4& ra1, float4& rb1,
                                            float4& ra2, float4& rb2, float4& ra3, float4& rb3) {
    wgrad_piece(ws, wn, p0, p_end, t, rows, a_row0, b_row0, ra0, rb0);
    wgrad_piece(ws, wn, p0, p_end, t + kBlock, rows, a_row0, b_row0, ra1, rb1);
    wgrad_piece(ws, wn, p0, p_end, t + 2 * kBlock, rows, a_row0, b_row0, ra2, rb2);
    wgrad_piece(ws, wn, p0, p_end, t + 3 * kBlock, rows, a_row0, b_row0, ra3, rb3);
}
__device__ __forceinline__ void wgrad_store(float (*A)[65], float (*B)[65], int t, int j,
                                            const float4& ra, const float4& rb) {
    const int idx = t + kBlock * j;
    const int r = idx >> 4, c = (idx & 15) * 4;
    A[r][c] = ra.x;
    A[r][c + 1] = ra.y;
    A[r][c + 2] = ra.z;
    A[r][c + 3] = ra.w;
    B[r][c] = rb.x;
    B[r][c + 1] = rb.y;
    B[r][c + 2] = rb.z;
    B[r][c + 3] = rb.w;
}

// Weight-gradient partials on the matrix cores: blockIdx.y picks the product
// (0: d1 x e -> W1, 1: d2 x h1 -> W2, 2: d3 x h2 -> W3), blockIdx.x a chunk
// of kChunk points; the workgroup's four wavefronts form the 64 x 64
// partial as four 32 x 32 tiles with v_mfma_f32_32x32x2f32, the points being
// the reduction dimension, two per instruction.  Operands are staged
// through LDS in tiles of 64 points by the whole workgroup (32-point tiles:
// 7 % slower); with VEC (rows 16-byte aligned: n a multiple of 4) each
// thread reads its share of a tile as 16-byte loads, the next tile's loads
// issued before the current tile's products.  Lane layout of that
// instruction: lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32];
// accumulator register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_hg_wgrad(const float* __restrict__ ws, int64_t wn,
                                                     int64_t n, float* __restrict__ part) {
    constexpr int kTile = 64;
    __shared__ float A[64][kTile + 1];
    __shared__ float B[64][kTile + 1];
    const int mat = blockIdx.y;
    const int rows = mat == 2 ? kOut : 64;
    const int a_row0 = mat == 0 ? 192 : mat == 1 ? 256 : 320;
    const int b_row0 = mat == 0 ? 0 : mat == 1 ? 64 : 128;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int ti = wave >> 1, tj = wave & 1;   // this wavefront's 32 x 32 tile
    const int li = lane % 32, lk = lane / 32;
    // the rows of A beyond `rows` are zero: a tile of them adds nothing
    const bool live_tile = 32 * ti < rows;
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int64_t p_begin = (int64_t)blockIdx.x * kChunk;
    const int64_t p_end = std::min<int64_t>(n, p_begin + kChunk);
    if (VEC) {
        // thread t stages four 4-point pieces of each operand per tile:
        // piece j is row (t + 256 j) / 16, points 4 ((t + 256 j) % 16) .. + 3
        float4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
        wgrad_fetch(ws, wn, p_begin, p_end, t, rows, a_row0, b_row0, ra0, rb0, ra1, rb1, ra2, rb2, ra3, rb3);
        for (int64_t p0 = p_begin; p0 < p_end; p0 += kTile) {
            wgrad_store(A, B, t, 0, ra0, rb0);
            wgrad_store(A, B, t, 1, ra1, rb1);
            wgrad_store(A, B, t, 2, ra2, rb2);
            wgrad_store(A, B, t, 3, ra3, rb3);
            __syncthreads();
            if (p0 + kTile < p_end)
                wgrad_fetch(ws, wn, p0 + kTile, p_end, t, rows, a_row0, b_row0, ra0, rb0, ra1, rb1,
                            ra2, rb2, ra3, rb3);
            if (live_tile) {
#pragma unroll
                for (int k0 = 0; k0 < kTile; k0 += 2)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[32 * ti + li][k0 + lk],
                                                               B[32 * tj + li][k0 + lk], acc, 0, 0, 0);
            }
            __syncthreads();
        }
    } else {
        for (int64_t p0 = p_begin; p0 < p_end; p0 += kTile) {
            // the workgroup stages 64 rows x 64 points of each operand
            // (coalesced along points)
            for (int idx = t; idx < 64 * kTile; idx += kBlock) {
                const int r = idx / kTile, c = idx % kTile;
                const int64_t pp = p0 + c;
                const bool in = pp < p_end;
                A[r][c] = (in && r < rows) ? ws[(int64_t)(a_row0 + r) * wn + pp] : 0.0f;
                B[r][c] = in ? ws[(int64_t)(b_row0 + r) * wn + pp] : 0.0f;
            }
            __syncthreads();
            if (live_tile) {
#pragma unroll
                for (int k0 = 0; k0 < kTile; k0 += 2)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[32 * ti + li][k0 + lk],
                                                               B[32 * tj + li][k0 + lk], acc, 0, 0, 0);
            }
            __syncthreads();
        }
    }
    float* out = part + ((int64_t)mat * gridDim.x + blockIdx.x) * 4096;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 32 * ti + 8 * (r / 4) + 4 * lk + (r % 4);
        const int j = 32 * tj + li;
        out[i * 64 + j] = acc[r];
    }
}

// gparams[weights] += the partials summed in chunk order.
__global__ __launch_bounds__(kBlock) void k_hg_wreduce(const float* __restrict__ part,
                                                       int64_t n_chunks,
                                                       float* __restrict__ gparams) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= kWeights) return;
    int mat, r;
    if (j < kW1) { mat = 0; r = j; }
    else if (j < kW1 + kW2) { mat = 1; r = j - kW1; }
    else { mat = 2; r = j - kW1 - kW2; }
    // chunk order; four partials' loads in flight at a time
    const float* src = part + (int64_t)mat * n_chunks * 4096 + r;
    float s = 0.0f;
    int64_t c = 0;
    for (; c + 4 <= n_chunks; c += 4) {
        const float a = src[c * 4096], b = src[(c + 1) * 4096], d = src[(c + 2) * 4096],
                    e = src[(c + 3) * 4096];
        s = (((s + a) + b) + d) + e;
    }
    for (; c < n_chunks; ++c) s += src[c * 4096];
    gparams[kTable + j] += s;
}

int grid_points(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

int check_hg(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

// (params may be NULL for the plan, which reads only positions)
int make_args(const float* params, const float* pos, int64_t ps, int64_t n, const float* lo,
              const float* hi, HgArgs& a, bool need_params = true) {
    if ((need_params && !params) || !pos || !lo || !hi) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FIPT_EINVAL, "n must be in [1, 2^31)");
    if (ps < n) return fail(FIPT_EINVAL, "pos_stride < n");
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(hi[k] > lo[k]))
            return fail(FIPT_EINVAL, "the box must be finite with bmin < bmax on every axis");
        a.lo[k] = lo[k];
        a.inv[k] = 1.0f / (hi[k] - lo[k]);
        if (!std::isfinite(a.inv[k])) return fail(FIPT_EINVAL, "the box is too thin");
    }
    a.params = params;
    a.pos = pos;
    a.ps = ps;
    a.n = n;
    return FIPT_OK;
}

// Lanes per slot of a level's table gather: the power of two nearest above
// a quarter of the mean list length of the level's (light, nonempty) slots,
// at most 64.
int lanes_per_slot(int64_t nnz, int64_t n_slots) {
    const int64_t mean = nnz / std::max<int64_t>(n_slots, 1);
    int L = 1;
    while (L < 64 && 4 * L < mean) L *= 2;
    return L;
}

// Slots of level l: the dense levels index (16 2^l + 1)^3 vertices.
int64_t level_slots(int l) {
    if (l < 3) {
        const int64_t r = (16 << l) + 1;
        return r * r * r;
    }
    return kT;
}

}  // namespace
}  // namespace fipt

struct fipt_hashgrid_plan_s {
    int32_t device = 0;
    int64_t n = 0;
    float lo[3], hi[3];
    float* pos = nullptr;                 // [3][n] device copy of the positions
    int2* ent[FIPT_HG_LEVELS] = {};       // per level: (p << 3 | corner, weight bits), by slot
    uint32_t* off[FIPT_HG_LEVELS] = {};   // per level: [2^19 + 1] slot ranges into ent
    uint32_t* heavy[FIPT_HG_LEVELS] = {}; // per level: the slots of more than kHeavy entries
    int64_t n_heavy[FIPT_HG_LEVELS] = {};
    int64_t nnz[FIPT_HG_LEVELS] = {};
    int lanes[FIPT_HG_LEVELS] = {};
};

using namespace fipt;

namespace {
void hg_plan_free(fipt_hashgrid_plan p) {
    if (!p) return;
    (void)hipFree(p->pos);
    for (int l = 0; l < FIPT_HG_LEVELS; ++l) {
        (void)hipFree(p->ent[l]);
        (void)hipFree(p->off[l]);
        (void)hipFree(p->heavy[l]);
    }
    delete p;
}
}  // namespace

extern "C" {

int64_t fipt_hashgrid_workspace_floats(int64_t n) {
    if (n < 1) return 0;
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    return (int64_t)(kWsRows + kFeatGradRows) * n + 3 * chunks * 4096;
}

int fipt_hashgrid_plan_create(const float* pos, int64_t pos_stride, int64_t n, const float* bmin_host,
                              const float* bmax_host, void* stream, fipt_hashgrid_plan* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    HgArgs a;
    int rc = make_args(nullptr, pos, pos_stride, n, bmin_host, bmax_host, a, false);
    if (rc) return rc;
    if (n >= (int64_t(1) << 28)) return fail(FIPT_EINVAL, "n must be below 2^28");
    hipStream_t st = (hipStream_t)stream;
    fipt_hashgrid_plan p = new fipt_hashgrid_plan_s();
    (void)hipGetDevice(&p->device);
    p->n = n;
    for (int k = 0; k < 3; ++k) {
        p->lo[k] = bmin_host[k];
        p->hi[k] = bmax_host[k];
    }
    const int64_t m = 8 * n;
    uint32_t *k_in = nullptr, *k_out = nullptr, *v_in = nullptr, *v_out = nullptr;
    unsigned long long* d_nnz = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    auto cleanup = [&]() {
        (void)hipFree(k_in);
        (void)hipFree(k_out);
        (void)hipFree(v_in);
        (void)hipFree(v_out);
        (void)hipFree(d_nnz);
        (void)hipFree(tmp);
    };
    auto bail = [&](int code, const char* what) {
        (void)hipStreamSynchronize(st);
        cleanup();
        hg_plan_free(p);
        return fail(code, "hashgrid plan: %s", what);
    };
    if (hipMalloc(reinterpret_cast<void**>(&p->pos), sizeof(float) * 3 * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k_in), sizeof(uint32_t) * m) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k_out), sizeof(uint32_t) * m) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&v_in), sizeof(uint32_t) * m) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&v_out), sizeof(uint32_t) * m) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d_nnz), sizeof(unsigned long long) * kLevels) != hipSuccess)
        return bail(FIPT_ENOMEM, "hipMalloc failed");
    for (int k = 0; k < 3; ++k)
        if (hipMemcpyAsync(p->pos + k * n, pos + k * pos_stride, sizeof(float) * n, hipMemcpyDeviceToDevice,
                           st) != hipSuccess)
            return bail(FIPT_EHIP, "copying the positions failed");
    a.pos = p->pos;
    a.ps = n;
    if (hipMemsetAsync(d_nnz, 0, sizeof(unsigned long long) * kLevels, st) != hipSuccess)
        return bail(FIPT_EHIP, "hipMemsetAsync failed");
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k_in, k_out, v_in, v_out, (int)m, 0, 20, st) !=
            hipSuccess ||
        hipMalloc(&tmp, tmp_bytes) != hipSuccess)
        return bail(FIPT_ENOMEM, "radix sort scratch");
    for (int l = 0; l < kLevels; ++l) {
        hipLaunchKernelGGL(k_hgp_keys, dim3(grid_points(n)), dim3(kBlock), 0, st, a, l, k_in, v_in,
                           d_nnz + l);
        if (hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k_in, k_out, v_in, v_out, (int)m, 0, 20, st) !=
            hipSuccess)
            return bail(FIPT_EHIP, "radix sort failed");
        // the nonzero count sizes the level's entry list
        unsigned long long h_nnz = 0;
        if (hipMemcpyAsync(&h_nnz, d_nnz + l, sizeof(h_nnz), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return bail(FIPT_EHIP, "counting the entries failed");
        p->nnz[l] = (int64_t)h_nnz;
        if (hipMalloc(reinterpret_cast<void**>(&p->ent[l]), sizeof(int2) * std::max<int64_t>(p->nnz[l], 1)) !=
                hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&p->off[l]), sizeof(uint32_t) * (kT + 1)) != hipSuccess)
            return bail(FIPT_ENOMEM, "hipMalloc entries failed");
        if (p->nnz[l] > 0)
            hipLaunchKernelGGL(k_hgp_entries, dim3(grid_points(p->nnz[l])), dim3(kBlock), 0, st, a, l, v_out,
                               p->nnz[l], p->ent[l]);
        hipLaunchKernelGGL(k_hgp_offsets, dim3(grid_points(kT + 1)), dim3(kBlock), 0, st, k_out, p->nnz[l],
                           p->off[l]);
        // slots of more than kHeavy entries get a workgroup each; the others
        // share lanes by the mean length of their lists
        const int64_t slots = level_slots(l);
        std::vector<uint32_t> h_off(slots + 1);
        if (hipMemcpyAsync(h_off.data(), p->off[l], sizeof(uint32_t) * (slots + 1), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return bail(FIPT_EHIP, "reading the slot ranges failed");
        std::vector<uint32_t> heavy;
        int64_t light_n = 0, light_slots = 0;
        for (int64_t q = 0; q < slots; ++q) {
            const uint32_t c = h_off[q + 1] - h_off[q];
            if (c > kHeavy) {
                heavy.push_back((uint32_t)q);
            } else if (c > 0) {
                light_n += c;
                ++light_slots;
            }
        }
        p->lanes[l] = lanes_per_slot(light_n, light_slots);
        p->n_heavy[l] = (int64_t)heavy.size();
        if (hipMalloc(reinterpret_cast<void**>(&p->heavy[l]), sizeof(uint32_t) * std::max<size_t>(heavy.size(), 1)) !=
            hipSuccess)
            return bail(FIPT_ENOMEM, "hipMalloc heavy slots failed");
        if (!heavy.empty() && hipMemcpyAsync(p->heavy[l], heavy.data(), sizeof(uint32_t) * heavy.size(),
                                             hipMemcpyHostToDevice, st) != hipSuccess)
            return bail(FIPT_EHIP, "copying the heavy slots failed");
        if (hipStreamSynchronize(st) != hipSuccess) return bail(FIPT_EHIP, "building a level failed");
    }
    if (check_hg("hashgrid plan") != FIPT_OK || hipStreamSynchronize(st) != hipSuccess)
        return bail(FIPT_EHIP, "building the entry lists failed");
    cleanup();
    *out = p;
    return FIPT_OK;
}

int fipt_hashgrid_plan_destroy(fipt_hashgrid_plan p) {
    clear_error();
    if (!p) return FIPT_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    hg_plan_free(p);
    if (prev >= 0) (void)hipSetDevice(prev);
    return FIPT_OK;
}

int fipt_hashgrid_forward(const float* params, const float* pos, int64_t pos_stride, int64_t n,
                          const float* bmin_host, const float* bmax_host, float* material,
                          int64_t mat_stride, void* stream) {
    clear_error();
    HgArgs a;
    int rc = make_args(params, pos, pos_stride, n, bmin_host, bmax_host, a);
    if (rc) return rc;
    if (!material) return fail(FIPT_EINVAL, "material is NULL");
    if (mat_stride < n) return fail(FIPT_EINVAL, "mat_stride < n");
    hipLaunchKernelGGL(k_hg_forward<false>, dim3(grid_points(n)), dim3(kBlock), 0, (hipStream_t)stream, a,
                       material, mat_stride, nullptr, 0);
    return check_hg("hashgrid_forward");
}

int fipt_hashgrid_forward_save(const float* params, const float* pos, int64_t pos_stride, int64_t n,
                               const float* bmin_host, const float* bmax_host, float* material,
                               int64_t mat_stride, float* workspace, int64_t workspace_floats,
                               void* stream) {
    clear_error();
    HgArgs a;
    int rc = make_args(params, pos, pos_stride, n, bmin_host, bmax_host, a);
    if (rc) return rc;
    if (!material || !workspace) return fail(FIPT_EINVAL, "NULL argument");
    if (mat_stride < n) return fail(FIPT_EINVAL, "mat_stride < n");
    if (workspace_floats < fipt_hashgrid_workspace_floats(n))
        return fail(FIPT_EINVAL, "workspace holds %lld floats, %lld needed", (long long)workspace_floats,
                    (long long)fipt_hashgrid_workspace_floats(n));
    hipLaunchKernelGGL(k_hg_forward<true>, dim3(grid_points(n)), dim3(kBlock), 0, (hipStream_t)stream, a,
                       material, mat_stride, workspace, n);
    return check_hg("hashgrid_forward_save");
}

static int hashgrid_backward(fipt_hashgrid_plan plan, const float* params, const float* grad_material,
                             int64_t gm_stride, float* grad_params, float* workspace,
                             int64_t workspace_floats, bool saved, void* stream) {
    if (!plan) return fail(FIPT_EINVAL, "plan is NULL");
    const int64_t n = plan->n;
    HgArgs a;
    int rc = make_args(params, plan->pos, n, n, plan->lo, plan->hi, a);
    if (rc) return rc;
    if (!grad_material || !grad_params || !workspace) return fail(FIPT_EINVAL, "NULL argument");
    if (gm_stride < n) return fail(FIPT_EINVAL, "gm_stride < n");
    if (workspace_floats < fipt_hashgrid_workspace_floats(n))
        return fail(FIPT_EINVAL, "workspace holds %lld floats, %lld needed", (long long)workspace_floats,
                    (long long)fipt_hashgrid_workspace_floats(n));
    hipStream_t st = (hipStream_t)stream;
    float2* fgrad = reinterpret_cast<float2*>(workspace + (int64_t)kWsRows * n);
    if (saved)
        hipLaunchKernelGGL(k_hg_backward<true>, dim3(grid_points(n)), dim3(kBlock), 0, st, a, grad_material,
                           gm_stride, workspace, n, fgrad);
    else
        hipLaunchKernelGGL(k_hg_backward<false>, dim3(grid_points(n)), dim3(kBlock), 0, st, a, grad_material,
                           gm_stride, workspace, n, fgrad);
    rc = check_hg("hashgrid_backward");
    if (rc) return rc;
    for (int l = 0; l < kLevels; ++l) {
        if (plan->nnz[l] == 0) continue;
        const int64_t slots = level_slots(l);
        const int L = plan->lanes[l];
        hipLaunchKernelGGL(k_hg_table_grad, dim3((unsigned)((slots * L + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, st, plan->ent[l], plan->off[l], fgrad + (int64_t)l * n, slots, L,
                           grad_params + (int64_t)l * kT * kFeat);
        if (plan->n_heavy[l] > 0)
            hipLaunchKernelGGL(k_hg_table_grad_heavy, dim3((unsigned)plan->n_heavy[l]), dim3(kBlock), 0, st,
                               plan->ent[l], plan->off[l], plan->heavy[l], fgrad + (int64_t)l * n,
                               grad_params + (int64_t)l * kT * kFeat);
    }
    rc = check_hg("hashgrid_table_grad");
    if (rc) return rc;
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    float* part = workspace + (int64_t)(kWsRows + kFeatGradRows) * n;
    // 16-byte staging when every workspace row starts 16-byte aligned
    const bool vec = (n % 4 == 0) && (reinterpret_cast<uintptr_t>(workspace) % 16 == 0);
    if (vec)
        hipLaunchKernelGGL(k_hg_wgrad<true>, dim3((unsigned)chunks, 3), dim3(kBlock), 0, st, workspace, n,
                           n, part);
    else
        hipLaunchKernelGGL(k_hg_wgrad<false>, dim3((unsigned)chunks, 3), dim3(kBlock), 0, st, workspace, n,
                           n, part);
    rc = check_hg("hashgrid_wgrad");
    if (rc) return rc;
    hipLaunchKernelGGL(k_hg_wreduce, dim3((kWeights + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       part, chunks, grad_params);
    return check_hg("hashgrid_wreduce");
}

int fipt_hashgrid_backward(fipt_hashgrid_plan plan, const float* params, const float* grad_material,
                           int64_t gm_stride, float* grad_params, float* workspace,
                           int64_t workspace_floats, void* stream) {
    clear_error();
    return hashgrid_backward(plan, params, grad_material, gm_stride, grad_params, workspace,
                             workspace_floats, false, stream);
}

int fipt_hashgrid_backward_saved(fipt_hashgrid_plan plan, const float* params,
                                 const float* grad_material, int64_t gm_stride, float* grad_params,
                                 float* workspace, int64_t workspace_floats, void* stream) {
    clear_error();
    return hashgrid_backward(plan, params, grad_material, gm_stride, grad_params, workspace,
                             workspace_floats, true, stream);
}

}  // extern "C"
