// HIP kernels of the factored re-render (Eq. 5 with the roughness lerp of
// Eq. 8), the photometric loss (Eq. 2 / Eq. 15) with its hand-written
// gradient, and the trilinear material grid with its adjoint, for gfx950.
//
// All of these are streaming kernels bound by HBM bandwidth: one thread per
// point, structure-of-arrays planes so every load and store of a wavefront
// is one contiguous 256-byte segment.  Storage is float32; the render-loss
// arithmetic runs in float64 (free at this arithmetic intensity).  The loss is summed per thread in
// double, reduced per workgroup in a fixed butterfly order and finally
// summed over workgroups in index order by one workgroup, so it is bitwise
// reproducible for a given point count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>
#include <vector>

#include "fipt_internal.hpp"

// Per-workgroup loss partials of fipt_render_loss_noalloc: one double per
// workgroup of the render-loss grid, which is capped at FIPT_LOSS_SLOTS - 1
// workgroups (each loops over its share of the points), so every point
// count fits.  Each GPU holds its own copy (16 KB) for the life of the
// process.  In host code the name is only a stand-in: the device address
// is looked up once per device (render_loss_scratch below) and only that
// address is handed to kernels.  Nothing in it needs clearing: every
// workgroup writes its own slot before the final sum reads it.
static __device__ __align__(256) double scratch[FIPT_LOSS_SLOTS - 1];

namespace fipt {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartials = FIPT_LOSS_SLOTS - 1;

struct SigmaTable {
    float s[FIPT_MAX_LEVELS];
    double inv_gap[FIPT_MAX_LEVELS];  // 1 / (s[j+1] - s[j])
};

// Tone maps in double: the per-point arithmetic of this kernel runs in
// float64, which removes the float32 cancellation in Lr - Lgt that would
// otherwise dominate the gradient of well-fit points.  The log-sRGB map
// Gamma(x) = sRGB-OETF(log(1 + x)) and its derivative share one log1p and
// one power, the power taken as exp(log(u) / 2.4) (a few ulp in double,
// and several times cheaper than a general pow).
template <int TONE>
__device__ __forceinline__ double tone_vd(double x, double& d) {
    if (TONE == 0) {
        d = 1.0;
        return x;
    }
    if (!(x > 0.0)) {
        d = 0.0;
        return 0.0;
    }
    const double u = log1p(x);
    if (u <= 0.0031308) {
        d = 12.92 / (1.0 + x);
        return 12.92 * u;
    }
    const double p = exp(log(u) * (1.0 / 2.4));
    d = (1.055 / 2.4) * p / (u * (1.0 + x));
    return 1.055 * p - 0.055;
}
template <int TONE>
__device__ __forceinline__ double tone(double x) {
    double d;
    return tone_vd<TONE>(x, d);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) t += sh[i];
    return t;
}

// Arguments of the render-loss kernel.  The masked form (Eq. 12 / 15 with
// the diffuse prior of Eq. 17) additionally reads the emission mask alpha
// (NULL: zero everywhere), writes d loss / d alpha when galpha is not NULL,
// and lets grad be NULL.
struct RLArgs {
    const float* sh;
    int64_t ss;
    int64_t n;
    int K;
    const float* mat;
    int64_t ms;
    const float* obs;
    int64_t os;
    double* partials;
    float* grad;
    int64_t gs;
    float* Lr;
    int64_t ls;
    const float* alpha;
    float* galpha;
    double lam;  // lambda_d of the diffuse prior
};

__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// MASK selects the masked loss with the prior: the compared value is
// (1 - alpha) Lr + alpha Lgt, whose derivative carries a factor (1 - alpha)
// into the material gradient, and lambda_d (|1 - sigma| + |m|) is added per
// point (derivative sign(0) = 0 at the kinks).  With alpha = 0 and
// lambda_d = 0 every operation it adds is exact, so it reproduces the plain
// loss bit for bit.
// Material, observation and loss of one point: the factored render of
// Eq. 5 with the lerp of Eq. 8, the squared tone-mapped residual of Eq. 2 /
// Eq. 15 and, with GRAD, d loss / d material into g5 (the roughness entry
// zero where sigma is clamped to the table) and, with MASK, d loss / d alpha.
// Shared by the plain render-loss kernel and the fused grid kernel, so both
// give the same bits for the same inputs.
template <int TONE, bool GRAD, bool MASK>
__device__ __forceinline__ double point_loss(const double (&a)[3], float sg, double m, double al,
                                             const float* sh, int64_t ss, int64_t p, int K,
                                             const float* obs, int64_t os, const SigmaTable& tab,
                                             double lam, double (&g5)[5], double& dal,
                                             double (&lr)[3]) {
    // bracket: largest j with s_j <= sigma, clamped to [0, K-2]
    int j = 0;
    for (int k = 1; k < K - 1; ++k) j = (tab.s[k] <= sg) ? k : j;
    const bool clamped = (sg < tab.s[0]) | (sg > tab.s[K - 1]);
    const double t = fmin(fmax(((double)sg - (double)tab.s[j]) * tab.inv_gap[j], 0.0), 1.0);
    const float* s0j = sh + (3 + 3 * j) * ss + p;
    const float* s1j = sh + (3 + 3 * K + 3 * j) * ss + p;
    double dsig = 0.0, dm = 0.0;
    double l = 0.0;
    dal = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double ld = sh[c * ss + p];
        const double A0 = s0j[c * ss], B0 = s0j[(c + 3) * ss];
        const double A1 = s1j[c * ss], B1 = s1j[(c + 3) * ss];
        const double L0 = (1.0 - t) * A0 + t * B0;
        const double L1 = (1.0 - t) * A1 + t * B1;
        const double kd = a[c] * (1.0 - m);
        const double ks = 0.04 * (1.0 - m) + a[c] * m;
        const double r = kd * ld + ks * L0 + L1;
        lr[c] = r;
        const double y = obs[c * os + p];
        const double h = MASK ? (1.0 - al) * r + al * y : r;
        double dh;
        const double res = tone_vd<TONE>(h, dh) - tone<TONE>(y);
        l += res * res;
        if (GRAD) {
            const double gh = 2.0 * res * dh;
            const double gr = MASK ? gh * (1.0 - al) : gh;
            g5[c] = gr * ((1.0 - m) * ld + m * L0);
            dm += gr * (-a[c] * ld + (a[c] - 0.04) * L0);
            dsig += gr * (ks * (B0 - A0) + (B1 - A1));
            if (MASK) dal += gh * (y - r);
        }
    }
    if (MASK) l += lam * (fabs(1.0 - (double)sg) + fabs(m));
    if (GRAD) {
        double gsig = clamped ? 0.0 : dsig * tab.inv_gap[j];
        if (MASK) {
            gsig += -lam * sgn(1.0 - (double)sg);
            dm += lam * sgn(m);
        }
        g5[3] = gsig;
        g5[4] = dm;
    }
    return l;
}

template <int TONE, bool GRAD, bool LR, bool MASK>
__global__ __launch_bounds__(kBlock) void k_render_loss(RLArgs g, SigmaTable tab) {
    __shared__ double s_red[kBlock / 64];
    const float* __restrict__ sh = g.sh;
    const float* __restrict__ mat = g.mat;
    const float* __restrict__ obs = g.obs;
    const int64_t ss = g.ss, ms = g.ms, os = g.os, n = g.n;
    const int K = g.K;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += stride) {
        const double a[3] = {mat[p], mat[ms + p], mat[2 * ms + p]};
        const float sg = mat[3 * ms + p];
        const double m = mat[4 * ms + p];
        const double al = (MASK && g.alpha) ? (double)g.alpha[p] : 0.0;
        double g5[5], lr[3], dal;
        acc += point_loss<TONE, GRAD, MASK>(a, sg, m, al, sh, ss, p, K, obs, os, tab, g.lam, g5,
                                            dal, lr);
        if (GRAD && (!MASK || g.grad)) {
            float* __restrict__ grad = g.grad;
            const int64_t gs = g.gs;
#pragma unroll
            for (int c = 0; c < 5; ++c) grad[c * gs + p] = (float)g5[c];
        }
        if (GRAD && MASK && g.galpha) g.galpha[p] = (float)dal;
        if (LR) {
            g.Lr[p] = (float)lr[0];
            g.Lr[g.ls + p] = (float)lr[1];
            g.Lr[2 * g.ls + p] = (float)lr[2];
        }
    }
    const double tot = block_sum(acc, s_red);
    if (threadIdx.x == 0) g.partials[blockIdx.x] = tot;
}

// Sum the per-workgroup partials in index order (one workgroup).
__global__ __launch_bounds__(kBlock) void k_final_sum(const double* partials, int n,
                                                      double* out) {
    __shared__ double s_red[kBlock / 64];
    // each thread sums a fixed contiguous run, then the fixed butterfly
    const int per = (n + kBlock - 1) / kBlock;
    double v = 0.0;
    for (int i = threadIdx.x * per; i < min(n, (int)(threadIdx.x + 1) * per); ++i) v += partials[i];
    const double tot = block_sum(v, s_red);
    if (threadIdx.x == 0) *out = tot;
}

// ---- trilinear grid --------------------------------------------------------
// Grid coordinates and weights are computed in float64: both grid kernels
// are bound by memory traffic, and float32 coordinates would carry an
// absolute error of ~1e-5 in the cell fraction (about one unit in the last
// place of res - 1).
struct GridFrame {
    double lo[3];
    double scale[3];   // (res - 1) / (bmax - bmin)
    int res;
};

__device__ __forceinline__ double grid_u(const GridFrame& g, float x, int axis) {
    return fmin(fmax(((double)x - g.lo[axis]) * g.scale[axis], 0.0), (double)(g.res - 1));
}

// Cell and trilinear weights of a point: `base` indexes the cell's lower
// corner in a grid plane, w[c] the weight of corner c (bit 0 x, bit 1 y,
// bit 2 z).
__device__ __forceinline__ int64_t grid_cell(const GridFrame& g, float x, float y, float z,
                                             double (&w)[8]) {
    const double ux = grid_u(g, x, 0), uy = grid_u(g, y, 1), uz = grid_u(g, z, 2);
    const int i = min((int)floor(ux), g.res - 2);
    const int j = min((int)floor(uy), g.res - 2);
    const int k = min((int)floor(uz), g.res - 2);
    const double fx = ux - i, fy = uy - j, fz = uz - k;
    w[0] = (1 - fx) * (1 - fy) * (1 - fz);
    w[1] = fx * (1 - fy) * (1 - fz);
    w[2] = (1 - fx) * fy * (1 - fz);
    w[3] = fx * fy * (1 - fz);
    w[4] = (1 - fx) * (1 - fy) * fz;
    w[5] = fx * (1 - fy) * fz;
    w[6] = (1 - fx) * fy * fz;
    w[7] = fx * fy * fz;
    const int64_t R = g.res;
    return i + R * (j + R * (int64_t)k);
}

// Trilinear value of one grid plane G at the cell `base` with weights w.
__device__ __forceinline__ double grid_value(const float* __restrict__ G, int64_t R,
                                             const double (&w)[8]) {
    const int64_t dy = R, dz = R * R;
    return w[0] * G[0] + w[1] * G[1] + w[2] * G[dy] + w[3] * G[dy + 1] + w[4] * G[dz] +
           w[5] * G[dz + 1] + w[6] * G[dz + dy] + w[7] * G[dz + dy + 1];
}

__global__ __launch_bounds__(kBlock) void k_grid_gather(const float* __restrict__ grid, int C,
                                                        GridFrame g, const float* __restrict__ pos,
                                                        int64_t ps, int64_t n,
                                                        float* __restrict__ out, int64_t os) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    double w[8];
    const int64_t base = grid_cell(g, pos[p], pos[ps + p], pos[2 * ps + p], w);
    const int64_t R = g.res;
    const int64_t plane = R * R * R;
    for (int c = 0; c < C; ++c) out[c * os + p] = (float)grid_value(grid + c * plane + base, R, w);
}

// Material fetch, factored render, loss and the per-column part of the
// adjoint fused, for the points of a grid plan in the plan's order (by node
// brick, cell, index).  The material of point q is the trilinear value of
// the five-channel grid at its position (the plan's record q), rounded to
// float as fipt_grid_gather stores it; loss and gradient are point_loss's.
// Each point's eight corner weights times its gradient (as stored, float)
// are summed over its column (at most kColumnMax consecutive points of one
// cell, never across a multiple of 16, so within one row of 16 lanes) by a
// segmented scan of three row shifts, and the column's last lane stores its
// 40 sums as one 160-byte record (channel-major, corners in order): the
// adjoint then reads one record per column instead of every point.  Products and sums are single precision (at most eight terms).
static_assert(kColumnMax <= 8, "the fused loss kernel's column scan takes three steps");

// v shifted down by d lanes within each row of 16 (0 where the source lies
// in the previous row).
template <int D>
__device__ __forceinline__ float row_shr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xF, 0xF, true));
}
template <int D>
__device__ __forceinline__ int32_t row_shr_i(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x110 + D, 0xF, 0xF, true);
}

template <int TONE, bool GP>
__device__ __forceinline__ void grid_render_loss(const GridPlanDev& P, const float* __restrict__ grid,
                                                 const GridFrame& gf, const float* __restrict__ sh,
                                                 int64_t ss, int K, const float* __restrict__ obs,
                                                 int64_t os, const SigmaTable& tab, double* partials,
                                                 float* __restrict__ gq, int64_t gqs) {
    __shared__ double s_red[kBlock / 64];
    const int64_t R = gf.res;
    const int64_t plane = R * R * R;
    const int64_t n = P.n_points;
    const int lane = threadIdx.x & 63;
    float* __restrict__ cs = P.csum;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // the loop runs over whole wavefronts (every lane takes part in the scan)
    for (int64_t q0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); q0 < n; q0 += stride) {
        const int64_t q = q0 + lane;
        const bool live = q < n;
        float wf[8], gf5[5];
        int32_t col1 = 0;   // home column + 1; 0 for no point
        if (live) {
            const float4 r = P.pts[q];
            double w[8];
            const int64_t base = grid_cell(gf, r.x, r.y, r.z, w);
            float mt[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) mt[c] = (float)grid_value(grid + c * plane + base, R, w);
            const double a[3] = {mt[0], mt[1], mt[2]};
            double g5[5], lr[3], dal;
            acc += point_loss<TONE, true, false>(a, mt[3], (double)mt[4], 0.0, sh, ss, q, K, obs, os,
                                                 tab, 0.0, g5, dal, lr);
#pragma unroll
            for (int c = 0; c < 5; ++c) gf5[c] = (float)g5[c];
            if (GP) {
#pragma unroll
                for (int c = 0; c < 5; ++c) gq[c * gqs + q] = gf5[c];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) wf[c] = (float)w[c];
            col1 = P.colq[q] + 1;
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) wf[c] = 0.0f;
#pragma unroll
            for (int c = 0; c < 5; ++c) gf5[c] = 0.0f;
        }
        // segmented inclusive sums over runs of equal column (every lane
        // takes part in the shifts; a shift from the previous row reads 0)
        const bool t1 = row_shr_i<1>(col1) == col1, t2 = row_shr_i<2>(col1) == col1,
                   t4 = row_shr_i<4>(col1) == col1;
        const int32_t nxt = __builtin_amdgcn_update_dpp(0, col1, 0x101, 0xF, 0xF, true);  // row_shl:1
        const bool tail = live && ((lane & 15) == 15 || nxt != col1);
        const int64_t hc = col1 - 1;
        float4* __restrict__ rec = reinterpret_cast<float4*>(cs) + hc * 10;
#pragma unroll
        for (int h = 0; h < 10; ++h) {   // channel h / 2, corners 4 (h % 2) .. + 3
            const float g = gf5[h >> 1];
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k] = wf[4 * (h & 1) + k] * g;
                const float u1 = row_shr<1>(v[k]);
                v[k] += t1 ? u1 : 0.0f;
                const float u2 = row_shr<2>(v[k]);
                v[k] += t2 ? u2 : 0.0f;
                const float u4 = row_shr<4>(v[k]);
                v[k] += t4 ? u4 : 0.0f;
            }
            if (tail) rec[h] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
    const double tot = block_sum(acc, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Without the tone map the kernel fits 96 registers (5 wavefronts per SIMD,
// no spills); the log-sRGB form keeps the compiler's allocation.
#define FIPT_GRID_LOSS_ARGS                                                                    \
    GridPlanDev P, const float* __restrict__ grid, GridFrame gf, const float* __restrict__ sh, \
        int64_t ss, int K, const float* __restrict__ obs, int64_t os, SigmaTable tab,          \
        double* partials, float* __restrict__ gq, int64_t gqs
template <bool GP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5, 8))) void
k_grid_render_loss(FIPT_GRID_LOSS_ARGS) {
    grid_render_loss<0, GP>(P, grid, gf, sh, ss, K, obs, os, tab, partials, gq, gqs);
}
template <bool GP>
__global__ __launch_bounds__(kBlock) void k_grid_render_loss_log(FIPT_GRID_LOSS_ARGS) {
    grid_render_loss<1, GP>(P, grid, gf, sh, ss, K, obs, os, tab, partials, gq, gqs);
}

// dst[c][q] = src[c][index of plan point q]: per-point planes into the
// plan's order (one thread per point and plane).
__global__ __launch_bounds__(kBlock) void k_plan_permute(const float4* __restrict__ pts, int64_t n,
                                                         const float* __restrict__ src, int64_t ss,
                                                         int planes, float* __restrict__ dst,
                                                         int64_t ds) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const int64_t p = __float_as_int(pts[q].w);
    for (int c = (int)blockIdx.y; c < planes; c += (int)gridDim.y) dst[c * ds + q] = src[c * ss + p];
}

// Adjoint of the gather: one workgroup per work unit (at most kAdjUnit
// columns of one node brick; a brick with no columns is one empty unit).  Each thread sums one column (at most
// kColumnMax points of one cell, in point order) into the eight corners of
// its cell in double.  The column sums meet in the brick's nodes as 64-bit
// fixed-point integers: the unit's largest column sum m and its column count
// n fix a per-channel scale 2^(62 - E) with n m < 2^E, so no sum of rounded
// column sums can overflow, and integer addition makes the node sums
// independent of the order in which threads add them.  A brick's only unit
// writes the nodes; the units of a brick of several write their node sums in
// double to the plan's scratch, and a second kernel adds them in unit order.
// A node reached by a non-finite gradient is NaN.
#ifndef FIPT_ADJ_BATCH
#define FIPT_ADJ_BATCH 8
#endif
constexpr int kAdjBlock = kAdjUnit;
static_assert(kAdjBlock == kBlock, "block_sum and the loss partials assume one workgroup size");
constexpr int kAdjBatch = FIPT_ADJ_BATCH;   // point records requested together

template <int C>
__device__ __forceinline__ void column_sums(const GridPlanDev& P, const GridFrame& g, int2 col,
                                            int ci, int cj, int ck, const float* __restrict__ gp,
                                            int64_t gs, double (&s)[8][C]) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) s[c][ch] = 0.0;
    // kAdjBatch point records of the column, then all their gradients, are
    // requested before any is used (a short column's tail repeats its last
    // point, whose lines are already on their way)
    const int cnt = col.y & 31;
#pragma unroll
    for (int v0 = 0; v0 < kColumnMax; v0 += kAdjBatch) {
        if (v0 >= cnt) break;
        float4 r[kAdjBatch];
#pragma unroll
        for (int v = 0; v < kAdjBatch; ++v) r[v] = P.pts[col.x + min(v0 + v, cnt - 1)];
        float gv[kAdjBatch][C];
#pragma unroll
        for (int v = 0; v < kAdjBatch; ++v) {
            const int32_t pi = __float_as_int(r[v].w);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) gv[v][ch] = gp[ch * gs + pi];
        }
#pragma unroll
        for (int v = 0; v < kAdjBatch; ++v) {
            if (v0 + v < cnt) {
                const double fx = grid_u(g, r[v].x, 0) - ci, fy = grid_u(g, r[v].y, 1) - cj,
                             fz = grid_u(g, r[v].z, 2) - ck;
                const double wx[2] = {1 - fx, fx}, wy[2] = {1 - fy, fy}, wz[2] = {1 - fz, fz};
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const double w = wx[c & 1] * wy[(c >> 1) & 1] * wz[c >> 2];
#pragma unroll
                    for (int ch = 0; ch < C; ++ch) s[c][ch] += w * (double)gv[v][ch];
                }
            }
        }
    }
}

// A work unit's node sums out: a brick's only unit writes its nodes (zeros
// where nothing reached them), a unit of a brick of several writes its node
// sums in double to its scratch slot for the combine kernel.  Non-finite
// flags become NaN.
template <int C>
__device__ __forceinline__ void store_brick(const GridPlanDev& P, const int4& unit, int ox, int oy,
                                            int oz, const unsigned long long (*acc)[kBrickNodes],
                                            const unsigned* bad, const int* expo,
                                            float* __restrict__ out) {
    const int tid = threadIdx.x;
    if (unit.w >= 0) {
        double* dst = P.part + (int64_t)unit.w * 8 * kBrickNodes;
        for (int i = tid; i < kBrickNodes; i += kAdjBlock) {
            const unsigned f = bad[i];
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                dst[ch * kBrickNodes + i] = (f >> ch) & 1 ? __longlong_as_double(0x7ff8000000000000ll)
                                                          : ldexp((double)(long long)acc[ch][i], expo[ch] - 62);
        }
        return;
    }
    const int64_t R = P.res;
    const int64_t plane = R * R * R;
    for (int i = tid; i < kBrickNodes; i += kAdjBlock) {
        const int x = ox + i % kBrickX, y = oy + (i / kBrickX) % kBrickY,
                  z = oz + i / (kBrickX * kBrickY);
        if (x >= R || y >= R || z >= R) continue;
        const int64_t v = x + R * (y + R * (int64_t)z);
        const unsigned f = bad[i];
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            const double d = ldexp((double)(long long)acc[ch][i], expo[ch] - 62);
            out[ch * plane + v] = (f >> ch) & 1 ? __int_as_float(0x7fc00000) : (float)d;
        }
    }
}

template <int C>
__global__ __launch_bounds__(kAdjBlock) void k_grid_adjoint(GridPlanDev P, GridFrame g,
                                                            const float* __restrict__ gp, int64_t gs,
                                                            float* __restrict__ out) {
    __shared__ unsigned long long acc[C][kBrickNodes];
    __shared__ unsigned bad[kBrickNodes];
    __shared__ double wmax[kAdjBlock / 64][C];
    __shared__ int expo[C];
    const int tid = threadIdx.x;
    const int4 unit = P.units[blockIdx.x];
    const int64_t brick = unit.x;
    const int bx = (int)(brick % P.nb[0]), by = (int)((brick / P.nb[0]) % P.nb[1]),
              bz = (int)(brick / ((int64_t)P.nb[0] * P.nb[1]));
    const int ox = bx * kBrickX, oy = by * kBrickY, oz = bz * kBrickZ;
    for (int i = tid; i < kBrickNodes; i += kAdjBlock) {
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[ch][i] = 0;
        bad[i] = 0;
    }
    __syncthreads();
    const int32_t ci = unit.y + tid;
    const bool live = ci < unit.z;
    double s[8][C];
    double m[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) m[ch] = 0.0;
    int lx = 0, ly = 0, lz = 0;
    // the column's sums and their largest magnitude per channel over the
    // corners this brick owns; non-finite sums flag their nodes
    if (live) {
        const int2 col = P.cols[ci];
        lx = ((col.y >> 5) & 63) - 1;
        ly = ((col.y >> 11) & 63) - 1;
        lz = ((col.y >> 17) & 63) - 1;
        column_sums<C>(P, g, col, ox + lx, oy + ly, oz + lz, gp, gs, s);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int nx = lx + (c & 1), ny = ly + ((c >> 1) & 1), nz = lz + (c >> 2);
            if (nx < 0 || ny < 0 || nz < 0 || nx >= kBrickX || ny >= kBrickY || nz >= kBrickZ)
                continue;
            const int node = nx + kBrickX * (ny + kBrickY * nz);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const double a = fabs(s[c][ch]);
                if (a <= DBL_MAX) m[ch] = fmax(m[ch], a);
                else atomicOr(&bad[node], 1u << ch);
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
        double v = m[ch];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if ((tid & 63) == 0) wmax[tid >> 6][ch] = v;
    }
    __syncthreads();
    if (tid < C) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kAdjBlock / 64; ++w) v = fmax(v, wmax[w][tid]);
        int e = 0;
        // every node sum is at most (columns) * v in magnitude
        if (v > 0.0) (void)frexp(v * (double)(unit.z - unit.y), &e);
        expo[tid] = e;
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int nx = lx + (c & 1), ny = ly + ((c >> 1) & 1), nz = lz + (c >> 2);
            if (nx < 0 || ny < 0 || nz < 0 || nx >= kBrickX || ny >= kBrickY || nz >= kBrickZ)
                continue;
            const int node = nx + kBrickX * (ny + kBrickY * nz);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const double v = s[c][ch];
                if (v != 0.0 && fabs(v) <= DBL_MAX) {
                    const long long q = (long long)rint(ldexp(v, 62 - expo[ch]));
                    atomicAdd(&acc[ch][node], (unsigned long long)q);
                }
            }
        }
    }
    __syncthreads();
    store_brick<C>(P, unit, ox, oy, oz, acc, bad, expo, out);
}


// Adjoint from the column sums of the fused loss kernel: one workgroup per
// work unit (at most kAdjUnit columns of one brick, as k_grid_adjoint), each
// thread reading one column's 40 sums (float, via the column entry's home
// column) instead of summing its points; the largest magnitude per channel
// over the corners the brick owns fixes the unit's fixed-point scale, and
// the sums are added into the brick's nodes as 64-bit integers.
// The launch has one workgroup more than units: the last sums the loss
// kernel's per-workgroup partials in index order (as k_final_sum).
__global__ __launch_bounds__(kAdjBlock) void k_grid_adjoint_sums(GridPlanDev P,
                                                                 float* __restrict__ out,
                                                                 const double* partials, int n_part,
                                                                 double* loss) {
    constexpr int C = 5;
    __shared__ unsigned long long acc[C][kBrickNodes];
    __shared__ unsigned bad[kBrickNodes];
    __shared__ float wmax[kAdjBlock / 64][C];
    __shared__ int expo[C];
    const int tid = threadIdx.x;
    if (blockIdx.x == gridDim.x - 1) {
        const int per = (n_part + kAdjBlock - 1) / kAdjBlock;
        double t = 0.0;
        for (int i = tid * per; i < min(n_part, (tid + 1) * per); ++i) t += partials[i];
        const double tot = block_sum(t, reinterpret_cast<double*>(wmax));
        if (tid == 0) *loss = tot;
        return;
    }
    const int4 unit = P.units[blockIdx.x];
    const int64_t brick = unit.x;
    const int bx = (int)(brick % P.nb[0]), by = (int)((brick / P.nb[0]) % P.nb[1]),
              bz = (int)(brick / ((int64_t)P.nb[0] * P.nb[1]));
    const int ox = bx * kBrickX, oy = by * kBrickY, oz = bz * kBrickZ;
    for (int i = tid; i < kBrickNodes; i += kAdjBlock) {
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[ch][i] = 0;
        bad[i] = 0;
    }
    const int32_t ci = unit.y + tid;
    const bool live = ci < unit.z;
    float v[8][C];
    float m[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) m[ch] = 0.0f;
    int lx = 0, ly = 0, lz = 0;
    if (live) {
        const int w = P.cols[ci].y;
        lx = ((w >> 5) & 63) - 1;
        ly = ((w >> 11) & 63) - 1;
        lz = ((w >> 17) & 63) - 1;
        const float4* rec = reinterpret_cast<const float4*>(P.csum) + (int64_t)P.hcol[ci] * 10;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            const float4 a = rec[2 * ch], b = rec[2 * ch + 1];
            v[0][ch] = a.x; v[1][ch] = a.y; v[2][ch] = a.z; v[3][ch] = a.w;
            v[4][ch] = b.x; v[5][ch] = b.y; v[6][ch] = b.z; v[7][ch] = b.w;
        }
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int nx = lx + (c & 1), ny = ly + ((c >> 1) & 1), nz = lz + (c >> 2);
            if (nx < 0 || ny < 0 || nz < 0 || nx >= kBrickX || ny >= kBrickY || nz >= kBrickZ)
                continue;
            const int node = nx + kBrickX * (ny + kBrickY * nz);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const float a = fabsf(v[c][ch]);
                if (a <= FLT_MAX) m[ch] = fmaxf(m[ch], a);
                else atomicOr(&bad[node], 1u << ch);
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
        float x = m[ch];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
        if ((tid & 63) == 0) wmax[tid >> 6][ch] = x;
    }
    __syncthreads();
    if (tid < C) {
        float x = 0.0f;
#pragma unroll
        for (int w = 0; w < kAdjBlock / 64; ++w) x = fmaxf(x, wmax[w][tid]);
        int e = 0;
        // every node sum is at most (columns) * x in magnitude
        if (x > 0.0f) (void)frexp((double)x * (double)(unit.z - unit.y), &e);
        expo[tid] = e;
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int nx = lx + (c & 1), ny = ly + ((c >> 1) & 1), nz = lz + (c >> 2);
            if (nx < 0 || ny < 0 || nz < 0 || nx >= kBrickX || ny >= kBrickY || nz >= kBrickZ)
                continue;
            const int node = nx + kBrickX * (ny + kBrickY * nz);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const float x = v[c][ch];
                if (x != 0.0f && fabsf(x) <= FLT_MAX) {
                    const long long q = (long long)rint(ldexp((double)x, 62 - expo[ch]));
                    atomicAdd(&acc[ch][node], (unsigned long long)q);
                }
            }
        }
    }
    __syncthreads();
    store_brick<C>(P, unit, ox, oy, oz, acc, bad, expo, out);
}

// The bricks of several units: their units' node sums added in unit order,
// one thread per (node, channel).
template <int C>
__global__ __launch_bounds__(kAdjBlock) void k_grid_adjoint_combine(GridPlanDev P, const int4* multi,
                                                                    float* __restrict__ out) {
    constexpr int kPer = (kBrickNodes * C + kAdjBlock - 1) / kAdjBlock;   // workgroups per brick
    const int4 mb = multi[blockIdx.x / kPer];
    const int j = (blockIdx.x % kPer) * kAdjBlock + threadIdx.x;   // ch * kBrickNodes + node
    if (j >= kBrickNodes * C) return;
    const int ch = j / kBrickNodes, i = j % kBrickNodes;
    const int64_t brick = mb.x;
    const int x = (int)(brick % P.nb[0]) * kBrickX + i % kBrickX,
              y = (int)((brick / P.nb[0]) % P.nb[1]) * kBrickY + (i / kBrickX) % kBrickY,
              z = (int)(brick / ((int64_t)P.nb[0] * P.nb[1])) * kBrickZ + i / (kBrickX * kBrickY);
    const int64_t R = P.res;
    if (x >= R || y >= R || z >= R) return;
    const double* src = P.part + (int64_t)mb.y * 8 * kBrickNodes + j;
    double t = 0.0;
    int u = 0;
    for (; u + 4 <= mb.z; u += 4) {
        const double a = src[(int64_t)u * 8 * kBrickNodes], b = src[(int64_t)(u + 1) * 8 * kBrickNodes],
                     c = src[(int64_t)(u + 2) * 8 * kBrickNodes], d = src[(int64_t)(u + 3) * 8 * kBrickNodes];
        t = (((t + a) + b) + c) + d;
    }
    for (; u < mb.z; ++u) t += src[(int64_t)u * 8 * kBrickNodes];
    out[(int64_t)ch * R * R * R + x + R * (y + R * (int64_t)z)] = (float)t;
}

__global__ void k_scale_by(const float* __restrict__ x, int64_t n, const double* __restrict__ f,
                           float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (float)((double)x[i] * f[0]);
}


int check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

template <int TONE, bool GRAD, bool LR, bool MASK>
void launch_rl(dim3 grid, hipStream_t st, const RLArgs& a, const SigmaTable& tab) {
    hipLaunchKernelGGL((k_render_loss<TONE, GRAD, LR, MASK>), grid, dim3(kBlock), 0, st, a, tab);
}

template <int TONE, bool GRAD, bool LR>
void launch_rl_mask(bool mask, dim3 grid, hipStream_t st, const RLArgs& a, const SigmaTable& tab) {
    if (mask) launch_rl<TONE, GRAD, LR, true>(grid, st, a, tab);
    else launch_rl<TONE, GRAD, LR, false>(grid, st, a, tab);
}

template <int TONE>
void launch_rl_tone(bool g, bool l, bool mask, dim3 grid, hipStream_t st, const RLArgs& a,
                    const SigmaTable& tab) {
    if (g && l) launch_rl_mask<TONE, true, true>(mask, grid, st, a, tab);
    else if (g) launch_rl_mask<TONE, true, false>(mask, grid, st, a, tab);
    else if (l) launch_rl_mask<TONE, false, true>(mask, grid, st, a, tab);
    else launch_rl_mask<TONE, false, false>(mask, grid, st, a, tab);
}

}  // namespace

int render_loss_scratch(double** out, int64_t* capacity) {
    // device addresses of `scratch`, one per GPU, looked up on first use
    // with that GPU current (the array's name is only a host-side stand-in)
    static std::mutex mu;
    static std::vector<double*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FIPT_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FIPT_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    *capacity = kMaxPartials;
    return FIPT_OK;
}

int render_loss_partials(int64_t n) {
    const int64_t want = (n + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, kMaxPartials));
}

int launch_render_loss(const float* sh, int64_t ss, int64_t n, int32_t K, const float* sigma,
                       const float* mat, int64_t ms, const float* obs, int64_t os, int32_t tone,
                       double* loss, double* partials, float* grad, int64_t gs, float* Lr,
                       int64_t ls, const RenderLossMask* mask, void* stream) {
    SigmaTable tab;
    for (int k = 0; k < FIPT_MAX_LEVELS; ++k) {
        tab.s[k] = k < K ? sigma[k] : 0.0f;
        tab.inv_gap[k] = (k + 1 < K) ? 1.0 / ((double)sigma[k + 1] - (double)sigma[k]) : 0.0;
    }
    const int blocks = render_loss_partials(n);
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(blocks);
    RLArgs a{sh, ss, n, K, mat, ms, obs, os, partials, grad, gs, Lr, ls,
             mask ? mask->alpha : nullptr, mask ? mask->grad_alpha : nullptr,
             mask ? mask->lambda_d : 0.0};
    const bool g = grad != nullptr || (mask && mask->grad_alpha), l = Lr != nullptr;
    if (tone == 0) launch_rl_tone<0>(g, l, mask != nullptr, grid, st, a, tab);
    else launch_rl_tone<1>(g, l, mask != nullptr, grid, st, a, tab);
    int rc = check("render_loss");
    if (rc) return rc;
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, st, partials, blocks, loss);
    return check("render_loss final sum");
}

int launch_scale_by(const float* x, int64_t n, const double* f, float* out, void* stream) {
    hipLaunchKernelGGL(k_scale_by, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, x, n, f, out);
    return check("scale_by");
}

static GridFrame make_frame(const float* bmin, const float* bmax, int R) {
    GridFrame g;
    for (int k = 0; k < 3; ++k) {
        g.lo[k] = bmin[k];
        g.scale[k] = (double)(R - 1) / ((double)bmax[k] - (double)bmin[k]);
    }
    g.res = R;
    return g;
}

int launch_grid_gather(const float* grid, int32_t C, int32_t R, const float* bmin,
                       const float* bmax, const float* pos, int64_t ps, int64_t n, float* out,
                       int64_t os, void* stream) {
    const GridFrame g = make_frame(bmin, bmax, R);
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_grid_gather, dim3((unsigned)blocks), dim3(kBlock), 0,
                       (hipStream_t)stream, grid, C, g, pos, ps, n, out, os);
    return check("grid_gather");
}

int launch_grid_scatter(const GridPlanDev& p, const float* gp, int32_t C, int64_t gs,
                        float* grad_grid, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const GridFrame g = make_frame(p.bmin, p.bmax, p.res);
    const dim3 nu((unsigned)p.n_units);
    const unsigned per = (unsigned)((kBrickNodes * C + kAdjBlock - 1) / kAdjBlock);
    switch (C) {
#define FIPT_SG(N)                                                                             \
    case N:                                                                                    \
        hipLaunchKernelGGL(k_grid_adjoint<N>, nu, dim3(kAdjBlock), 0, st, p, g, gp, gs, grad_grid); \
        if (p.n_multi > 0)                                                                     \
            hipLaunchKernelGGL(k_grid_adjoint_combine<N>, dim3((unsigned)(p.n_multi * per)), dim3(kAdjBlock), 0, st, p, p.multi, grad_grid); \
        break
        FIPT_SG(1); FIPT_SG(2); FIPT_SG(3); FIPT_SG(4);
        FIPT_SG(5); FIPT_SG(6); FIPT_SG(7); FIPT_SG(8);
#undef FIPT_SG
        default:
            return fail(FIPT_EINVAL, "channels must be in [1, 8]");
    }
    return check("grid_adjoint");
}

int launch_grid_render_loss(const GridPlanDev& p, const float* grid, const float* sh, int64_t ss,
                            int32_t K, const float* sigma, const float* obs, int64_t os,
                            int32_t tone, double* loss, double* partials, float* gq, int64_t gqs,
                            float* grad_grid, void* stream) {
    SigmaTable tab;
    for (int k = 0; k < FIPT_MAX_LEVELS; ++k) {
        tab.s[k] = k < K ? sigma[k] : 0.0f;
        tab.inv_gap[k] = (k + 1 < K) ? 1.0 / ((double)sigma[k + 1] - (double)sigma[k]) : 0.0;
    }
    hipStream_t st = (hipStream_t)stream;
    const GridFrame g = make_frame(p.bmin, p.bmax, p.res);
    const int blocks = render_loss_partials(p.n_points);
    const dim3 gr(blocks), bl(kBlock);
    if (tone == 0 && gq)
        hipLaunchKernelGGL(k_grid_render_loss<true>, gr, bl, 0, st, p, grid, g, sh, ss, K, obs, os, tab, partials, gq, gqs);
    else if (tone == 0)
        hipLaunchKernelGGL(k_grid_render_loss<false>, gr, bl, 0, st, p, grid, g, sh, ss, K, obs, os, tab, partials, gq, gqs);
    else if (gq)
        hipLaunchKernelGGL(k_grid_render_loss_log<true>, gr, bl, 0, st, p, grid, g, sh, ss, K, obs, os, tab, partials, gq, gqs);
    else
        hipLaunchKernelGGL(k_grid_render_loss_log<false>, gr, bl, 0, st, p, grid, g, sh, ss, K, obs, os, tab, partials, gq, gqs);
    int rc = check("grid_render_loss");
    if (rc) return rc;
    hipLaunchKernelGGL(k_grid_adjoint_sums, dim3((unsigned)p.n_units + 1), dim3(kAdjBlock), 0, st, p,
                       grad_grid, partials, blocks, loss);
    if (p.n_multi > 0) {
        const unsigned per = (unsigned)((kBrickNodes * 5 + kAdjBlock - 1) / kAdjBlock);
        hipLaunchKernelGGL(k_grid_adjoint_combine<5>, dim3((unsigned)(p.n_multi * per)), dim3(kAdjBlock),
                           0, st, p, p.multi, grad_grid);
    }
    return check("grid_render_loss adjoint");
}

int launch_plan_permute(const GridPlanDev& p, const float* src, int32_t planes, int64_t ss,
                        float* dst, int64_t ds, void* stream) {
    const int64_t n = p.n_points;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)std::min(planes, 64));
    hipLaunchKernelGGL(k_plan_permute, grid, dim3(kBlock), 0, (hipStream_t)stream, p.pts, n, src,
                       ss, planes, dst, ds);
    return check("plan_permute");
}

}  // namespace fipt
