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
// Forward: one thread per point (one point per thread and no grid-stride
// loop, so the compiler cannot hoist the weight reads out of a loop into
// registers); each workgroup copies the three weight matrices (34 KB) into
// LDS, and every thread of a workgroup reads the same weight at once (an
// LDS broadcast); the point's hidden activations stay in registers.  The 256 table gathers per point (8 vertices x 32 levels, 8
// bytes each) are the memory traffic; the tables (134 MB) live in HBM and
// the MALL.
//
// Backward: one thread per point recomputes the forward pass, back-propagates
// through the MLP, adds each feature gradient into the table entries of its
// 8 vertices per level with float atomics (the order of those additions, and
// so the last bits of the table gradient, depends on scheduling), and
// stores its activations and layer gradients in a workspace.  The weight
// gradients are sums over points of outer products (three small GEMMs with
// the point count as the reduction dimension): a split-K kernel forms one
// 64 x 64 partial per chunk of 8192 points on the matrix cores, and a final
// kernel adds the partials in chunk order, so weight gradients are
// reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

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
constexpr int kChunk = 8192;              // points per weight-gradient partial
constexpr int kWsRows = 3 * 64 + 2 * 64 + kOut;   // e, h1, h2, d1, d2, d3
constexpr int kAggregateLevels = 6;       // levels whose table updates are combined per wavefront

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

__device__ __forceinline__ void load_weights(const float* __restrict__ params, float* w) {
    for (int i = threadIdx.x; i < kWeights; i += kBlock) w[i] = params[kTable + i];
    __syncthreads();
}

// z1 = W1 e, level by level: each level's two features are folded into the
// 64 accumulators as soon as they are interpolated (and stored to ws_e when
// it is not NULL, rows 2l and 2l + 1).
__device__ __forceinline__ void encode_layer1(const float* __restrict__ tab, const float* W1,
                                              const float p[3], float z1[kHid],
                                              float* __restrict__ ws_e, int64_t wn) {
#pragma unroll
    for (int o = 0; o < kHid; ++o) z1[o] = 0.0f;
    const float2* t2 = reinterpret_cast<const float2*>(tab);
#pragma unroll 1
    for (int l = 0; l < kLevels; ++l) {
        uint32_t idx[8];
        float w[8];
        corners(l, p, idx, w);
        const float2* t = t2 + (int64_t)l * kT;
        float e0 = 0.0f, e1 = 0.0f;
        // from level 20 on (2^24 cells per axis and more) a single-precision
        // position sits exactly on a vertex: 7 of the 8 weights are zero, and
        // their reads are skipped
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (w[k] != 0.0f) {
                const float2 v = t[idx[k]];
                e0 = fmaf(w[k], v.x, e0);
                e1 = fmaf(w[k], v.y, e1);
            }
        }
        if (ws_e) {
            ws_e[(int64_t)(2 * l) * wn] = e0;
            ws_e[(int64_t)(2 * l + 1) * wn] = e1;
        }
#pragma unroll
        for (int o = 0; o < kHid; ++o)
            z1[o] = fmaf(W1[o * kIn + 2 * l + 1], e1, fmaf(W1[o * kIn + 2 * l], e0, z1[o]));
    }
}

// h = relu(W x) for 64 x 64 W, with a bit mask of the positive outputs.
__device__ __forceinline__ void dense_relu(const float* W, const float* x, float* h, uint64_t& pos) {
    pos = 0;
#pragma unroll
    for (int o = 0; o < kHid; ++o) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < kHid; ++i) s = fmaf(W[o * kHid + i], x[i], s);
        h[o] = fmaxf(s, 0.0f);
        pos |= (uint64_t)(s > 0.0f) << o;
        // one output at a time: keep the scheduler from hoisting the weight
        // reads of later outputs (it would spill them)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Table update of one vertex per lane, combined across the wavefront: lanes
// naming the same slot are summed by a butterfly and one of them adds the
// total.  On the coarse levels neighbouring pixels share vertices, and one
// atomic per distinct slot replaces up to 64 on the same address.
__device__ __forceinline__ void add_combined(float* t, uint32_t idx, float v0, float v1, int lane) {
    uint64_t todo = __builtin_amdgcn_ballot_w64(true);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t lidx = __shfl(idx, leader, 64);
        const bool mine = ((todo >> lane) & 1ull) && idx == lidx;
        todo &= ~__builtin_amdgcn_ballot_w64(mine);
        float s0 = mine ? v0 : 0.0f, s1 = mine ? v1 : 0.0f;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            s0 += __shfl_xor(s0, m, 64);
            s1 += __shfl_xor(s1, m, 64);
        }
        if (lane == leader) {
            atomicAdd(t + (int64_t)lidx * kFeat, s0);
            atomicAdd(t + (int64_t)lidx * kFeat + 1, s1);
        }
    }
}

// Occupancy targets keep the compiler from hoisting the weight loads of the
// unrolled products into hundreds of registers: 4 waves per SIMD (at most
// 128 VGPRs) for the forward pass, 3 (at most 168) for the backward pass,
// whose layer gradients hold two 64-vectors at once.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_hg_forward(HgArgs a, float* __restrict__ out,
                                                       int64_t os) {
    __shared__ float w[kWeights];
    load_weights(a.params, w);
    const float* W1 = w;
    const float* W2 = w + kW1;
    const float* W3 = w + kW1 + kW2;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < a.n) {
        float p[3], h1[kHid], h2[kHid];
        unit_pos(a, i, p);
        encode_layer1(a.params, W1, p, h1, nullptr, 0);
        uint64_t m1, m2;
#pragma unroll
        for (int o = 0; o < kHid; ++o) h1[o] = fmaxf(h1[o], 0.0f);
        dense_relu(W2, h1, h2, m2);
        (void)m1;
#pragma unroll
        for (int o = 0; o < kOut; ++o) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < kHid; ++j) s = fmaf(W3[o * kHid + j], h2[j], s);
            out[o * os + i] = 1.0f / (1.0f + expf(-s));
        }
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_hg_backward(HgArgs a, const float* __restrict__ gy,
                                                        int64_t gs, float* __restrict__ gparams,
                                                        float* __restrict__ ws, int64_t wn) {
    __shared__ float w[kWeights];
    load_weights(a.params, w);
    const float* W1 = w;
    const float* W2 = w + kW1;
    const float* W3 = w + kW1 + kW2;
    // every lane of a wavefront runs the body (the table updates combine
    // lanes); a lane past the last point takes the origin and adds zeros
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < a.n;
    const int lane = threadIdx.x & 63;
    {
        float p[3] = {0.0f, 0.0f, 0.0f}, h1[kHid], h2[kHid];
        if (live) unit_pos(a, i, p);
        encode_layer1(a.params, W1, p, h1, live ? ws + i : nullptr, wn);
        uint64_t m1 = 0, m2;
#pragma unroll
        for (int o = 0; o < kHid; ++o) {
            m1 |= (uint64_t)(h1[o] > 0.0f) << o;
            h1[o] = fmaxf(h1[o], 0.0f);
            if (live) ws[(int64_t)(64 + o) * wn + i] = h1[o];
        }
        dense_relu(W2, h1, h2, m2);
#pragma unroll
        for (int o = 0; o < kHid; ++o)
            if (live) ws[(int64_t)(128 + o) * wn + i] = h2[o];
        float d3[kOut];
#pragma unroll
        for (int o = 0; o < kOut; ++o) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < kHid; ++j) s = fmaf(W3[o * kHid + j], h2[j], s);
            const float y = 1.0f / (1.0f + expf(-s));
            d3[o] = live ? gy[o * gs + i] * y * (1.0f - y) : 0.0f;
            if (live) ws[(int64_t)(320 + o) * wn + i] = d3[o];
        }
        // d2 = (W3^T d3) masked, in h2's registers
#pragma unroll
        for (int j = 0; j < kHid; ++j) {
            float s = 0.0f;
#pragma unroll
            for (int o = 0; o < kOut; ++o) s = fmaf(W3[o * kHid + j], d3[o], s);
            h2[j] = ((m2 >> j) & 1ull) ? s : 0.0f;
            if (live) ws[(int64_t)(256 + j) * wn + i] = h2[j];
            __builtin_amdgcn_sched_barrier(0);
        }
        // d1 = (W2^T d2) masked, in h1's registers
#pragma unroll
        for (int k = 0; k < kHid; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < kHid; ++j) s = fmaf(W2[j * kHid + k], h2[j], s);
            h1[k] = ((m1 >> k) & 1ull) ? s : 0.0f;
            if (live) ws[(int64_t)(192 + k) * wn + i] = h1[k];
            __builtin_amdgcn_sched_barrier(0);
        }
        // per level: feature gradients (W1^T d1, rows 2l and 2l + 1) into the
        // table entries of the cell's 8 vertices
#pragma unroll 1
        for (int l = 0; l < kLevels; ++l) {
            float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
            for (int o = 0; o < kHid; ++o) {
                g0 = fmaf(W1[o * kIn + 2 * l], h1[o], g0);
                g1 = fmaf(W1[o * kIn + 2 * l + 1], h1[o], g1);
            }
            uint32_t idx[8];
            float wt[8];
            corners(l, p, idx, wt);
            float* t = gparams + (int64_t)l * kT * kFeat;
            if (l < kAggregateLevels) {
#pragma unroll
                for (int k = 0; k < 8; ++k) add_combined(t, idx[k], wt[k] * g0, wt[k] * g1, lane);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (live && wt[k] != 0.0f) {   // zero-weight vertices add nothing
                        atomicAdd(t + (int64_t)idx[k] * kFeat, wt[k] * g0);
                        atomicAdd(t + (int64_t)idx[k] * kFeat + 1, wt[k] * g1);
                    }
                }
            }
        }
    }
}

// Weight-gradient partials on the matrix cores: blockIdx.y picks the product
// (0: d1 x e -> W1, 1: d2 x h1 -> W2, 2: d3 x h2 -> W3), blockIdx.x a chunk
// of kChunk points; the workgroup's four wavefronts form the 64 x 64
// partial as four 32 x 32 tiles with v_mfma_f32_32x32x2f32, the points being
// the reduction dimension, two per instruction.  Operands are staged
// through LDS in tiles of 64 points by the whole workgroup (32-point tiles:
// 7 % slower).  Lane layout of that instruction: lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register r of lane l
// holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
typedef float v16f __attribute__((ext_vector_type(16)));

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
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int64_t p_begin = (int64_t)blockIdx.x * kChunk;
    const int64_t p_end = std::min<int64_t>(n, p_begin + kChunk);
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
#pragma unroll
        for (int k0 = 0; k0 < kTile; k0 += 2)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[32 * ti + li][k0 + lk],
                                                       B[32 * tj + li][k0 + lk], acc, 0, 0, 0);
        __syncthreads();
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
    float s = 0.0f;
    for (int64_t c = 0; c < n_chunks; ++c) s += part[((int64_t)mat * n_chunks + c) * 4096 + r];
    gparams[kTable + j] += s;
}

int grid_points(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

int check_hg(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

int make_args(const float* params, const float* pos, int64_t ps, int64_t n, const float* lo,
              const float* hi, HgArgs& a) {
    if (!params || !pos || !lo || !hi) return fail(FIPT_EINVAL, "NULL argument");
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

}  // namespace
}  // namespace fipt

using namespace fipt;

extern "C" {

int64_t fipt_hashgrid_workspace_floats(int64_t n) {
    if (n < 1) return 0;
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    return (int64_t)kWsRows * n + 3 * chunks * 4096;
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
    hipLaunchKernelGGL(k_hg_forward, dim3(grid_points(n)), dim3(kBlock), 0, (hipStream_t)stream, a,
                       material, mat_stride);
    return check_hg("hashgrid_forward");
}

int fipt_hashgrid_backward(const float* params, const float* pos, int64_t pos_stride, int64_t n,
                           const float* bmin_host, const float* bmax_host,
                           const float* grad_material, int64_t gm_stride, float* grad_params,
                           float* workspace, int64_t workspace_floats, void* stream) {
    clear_error();
    HgArgs a;
    int rc = make_args(params, pos, pos_stride, n, bmin_host, bmax_host, a);
    if (rc) return rc;
    if (!grad_material || !grad_params || !workspace) return fail(FIPT_EINVAL, "NULL argument");
    if (gm_stride < n) return fail(FIPT_EINVAL, "gm_stride < n");
    if (workspace_floats < fipt_hashgrid_workspace_floats(n))
        return fail(FIPT_EINVAL, "workspace holds %lld floats, %lld needed", (long long)workspace_floats,
                    (long long)fipt_hashgrid_workspace_floats(n));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_hg_backward, dim3(grid_points(n)), dim3(kBlock), 0, st, a, grad_material,
                       gm_stride, grad_params, workspace, n);
    rc = check_hg("hashgrid_backward");
    if (rc) return rc;
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    float* part = workspace + (int64_t)kWsRows * n;
    hipLaunchKernelGGL(k_hg_wgrad, dim3((unsigned)chunks, 3), dim3(kBlock), 0, st, workspace, n, n,
                       part);
    rc = check_hg("hashgrid_wgrad");
    if (rc) return rc;
    hipLaunchKernelGGL(k_hg_wreduce, dim3((kWeights + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       part, chunks, grad_params);
    return check_hg("hashgrid_wreduce");
}

}  // extern "C"
