// HIP kernels of the factored re-render (Eq. 5 with the roughness lerp of
// Eq. 8), the photometric loss (Eq. 2 / Eq. 15) with its hand-written
// gradient, and the trilinear material grid with its adjoint, for gfx950.
//
// All of these are streaming kernels bound by HBM bandwidth: one thread per
// point, structure-of-arrays planes so every load and store of a wavefront
// is one contiguous 256-byte segment.  The loss is summed per thread in
// double, reduced per workgroup in a fixed butterfly order and finally
// summed over workgroups in index order by one workgroup, so it is bitwise
// reproducible for a given point count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fipt_internal.hpp"

namespace fipt {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartials = FIPT_LOSS_SLOTS - 1;

struct SigmaTable {
    float s[FIPT_MAX_LEVELS];
    float inv_gap[FIPT_MAX_LEVELS];  // 1 / (s[j+1] - s[j])
};

__device__ __forceinline__ float srgb_oetf(float x) {
    return x <= 0.0031308f ? 12.92f * x : 1.055f * powf(x, 1.0f / 2.4f) - 0.055f;
}
__device__ __forceinline__ float srgb_oetf_d(float x) {
    return x <= 0.0031308f ? 12.92f : (1.055f / 2.4f) * powf(x, 1.0f / 2.4f - 1.0f);
}

template <int TONE>
__device__ __forceinline__ float tone(float x) {
    if (TONE == 0) return x;
    return srgb_oetf(log1pf(fmaxf(x, 0.0f)));
}
template <int TONE>
__device__ __forceinline__ float tone_d(float x) {
    if (TONE == 0) return 1.0f;
    if (!(x > 0.0f)) return 0.0f;
    return srgb_oetf_d(log1pf(x)) / (1.0f + x);
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

template <int TONE, bool GRAD, bool LR>
__global__ __launch_bounds__(kBlock) void k_render_loss(
    const float* __restrict__ sh, int64_t ss, int64_t n, int K, SigmaTable tab,
    const float* __restrict__ mat, int64_t ms, const float* __restrict__ obs, int64_t os,
    double* __restrict__ partials, float* __restrict__ grad, int64_t gs, float* __restrict__ Lr,
    int64_t ls) {
    __shared__ double s_red[kBlock / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += stride) {
        const float ar = mat[p], ag = mat[ms + p], ab = mat[2 * ms + p];
        const float sg = mat[3 * ms + p], m = mat[4 * ms + p];
        // bracket: largest j with s_j <= sigma, clamped to [0, K-2]
        int j = 0;
        for (int k = 1; k < K - 1; ++k) j = (tab.s[k] <= sg) ? k : j;
        const bool clamped = (sg < tab.s[0]) | (sg > tab.s[K - 1]);
        const float t = fminf(fmaxf((sg - tab.s[j]) * tab.inv_gap[j], 0.0f), 1.0f);
        const float ld[3] = {sh[p], sh[ss + p], sh[2 * ss + p]};
        const float* s0j = sh + (3 + 3 * j) * ss + p;
        const float* s1j = sh + (3 + 3 * K + 3 * j) * ss + p;
        float a[3] = {ar, ag, ab};
        float dsig = 0.0f, dm = 0.0f;
        float da[3];
        float lr[3];
        float l = 0.0f;
        for (int c = 0; c < 3; ++c) {
            const float A0 = s0j[c * ss], B0 = s0j[(c + 3) * ss];
            const float A1 = s1j[c * ss], B1 = s1j[(c + 3) * ss];
            const float L0 = A0 + t * (B0 - A0);
            const float L1 = A1 + t * (B1 - A1);
            const float kd = a[c] * (1.0f - m);
            const float ks = 0.04f * (1.0f - m) + a[c] * m;
            const float r = kd * ld[c] + ks * L0 + L1;
            lr[c] = r;
            const float y = obs[c * os + p];
            const float res = tone<TONE>(r) - tone<TONE>(y);
            l += res * res;
            if (GRAD) {
                const float g = 2.0f * res * tone_d<TONE>(r);
                da[c] = g * ((1.0f - m) * ld[c] + m * L0);
                dm += g * (-a[c] * ld[c] + (a[c] - 0.04f) * L0);
                dsig += g * (ks * (B0 - A0) + (B1 - A1));
            }
        }
        acc += (double)l;
        if (GRAD) {
            grad[p] = da[0];
            grad[gs + p] = da[1];
            grad[2 * gs + p] = da[2];
            grad[3 * gs + p] = clamped ? 0.0f : dsig * tab.inv_gap[j];
            grad[4 * gs + p] = dm;
        }
        if (LR) {
            Lr[p] = lr[0];
            Lr[ls + p] = lr[1];
            Lr[2 * ls + p] = lr[2];
        }
    }
    const double tot = block_sum(acc, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
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
struct GridFrame {
    float lo[3];
    float scale[3];   // (res - 1) / (bmax - bmin)
    int res;
};

__device__ __forceinline__ void cell_of(const GridFrame& g, float x, float y, float z, int& i,
                                        int& j, int& k, float& fx, float& fy, float& fz) {
    const float top = (float)(g.res - 1);
    const float ux = fminf(fmaxf((x - g.lo[0]) * g.scale[0], 0.0f), top);
    const float uy = fminf(fmaxf((y - g.lo[1]) * g.scale[1], 0.0f), top);
    const float uz = fminf(fmaxf((z - g.lo[2]) * g.scale[2], 0.0f), top);
    i = min((int)floorf(ux), g.res - 2);
    j = min((int)floorf(uy), g.res - 2);
    k = min((int)floorf(uz), g.res - 2);
    fx = ux - (float)i;
    fy = uy - (float)j;
    fz = uz - (float)k;
}

__global__ __launch_bounds__(kBlock) void k_grid_gather(const float* __restrict__ grid, int C,
                                                        GridFrame g, const float* __restrict__ pos,
                                                        int64_t ps, int64_t n,
                                                        float* __restrict__ out, int64_t os) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    int i, j, k;
    float fx, fy, fz;
    cell_of(g, pos[p], pos[ps + p], pos[2 * ps + p], i, j, k, fx, fy, fz);
    const int64_t R = g.res;
    const int64_t plane = R * R * R;
    const int64_t base = i + R * (j + R * (int64_t)k);
    const int64_t dy = R, dz = R * R;
    const float w000 = (1 - fx) * (1 - fy) * (1 - fz), w100 = fx * (1 - fy) * (1 - fz);
    const float w010 = (1 - fx) * fy * (1 - fz), w110 = fx * fy * (1 - fz);
    const float w001 = (1 - fx) * (1 - fy) * fz, w101 = fx * (1 - fy) * fz;
    const float w011 = (1 - fx) * fy * fz, w111 = fx * fy * fz;
    for (int c = 0; c < C; ++c) {
        const float* G = grid + c * plane + base;
        const float v = w000 * G[0] + w100 * G[1] + w010 * G[dy] + w110 * G[dy + 1] +
                        w001 * G[dz] + w101 * G[dz + 1] + w011 * G[dz + dy] +
                        w111 * G[dz + dy + 1];
        out[c * os + p] = v;
    }
}

// Adjoint, pass 1: per occupied cell, the eight corner sums of
// weight * gradient over the cell's points (taken in index order), double.
template <int C>
__global__ __launch_bounds__(kBlock) void k_scatter_cells(GridPlanDev plan, GridFrame g,
                                                          const float* __restrict__ gp,
                                                          int64_t gs) {
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= plan.n_occ) return;
    double acc[8][C];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[c][ch] = 0.0;
    const int64_t n = plan.n_points;
    const float* pos = plan.pos;
    // the plan fixed the cell; fractions are taken relative to it
    const int32_t cid = plan.cell_id[m];
    const int cr = g.res - 1;
    const int ci = cid % cr, cj = (cid / cr) % cr, ck = cid / (cr * cr);
    const float top = (float)(g.res - 1);
    for (int32_t q = plan.cell_start[m]; q < plan.cell_start[m + 1]; ++q) {
        const int32_t p = plan.perm[q];
        const float fx = fminf(fmaxf((pos[p] - g.lo[0]) * g.scale[0], 0.0f), top) - (float)ci;
        const float fy = fminf(fmaxf((pos[n + p] - g.lo[1]) * g.scale[1], 0.0f), top) - (float)cj;
        const float fz = fminf(fmaxf((pos[2 * n + p] - g.lo[2]) * g.scale[2], 0.0f), top) - (float)ck;
        const float w[8] = {(1 - fx) * (1 - fy) * (1 - fz), fx * (1 - fy) * (1 - fz),
                            (1 - fx) * fy * (1 - fz),       fx * fy * (1 - fz),
                            (1 - fx) * (1 - fy) * fz,       fx * (1 - fy) * fz,
                            (1 - fx) * fy * fz,             fx * fy * fz};
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            const double v = (double)gp[ch * gs + p];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c][ch] += (double)w[c] * v;
        }
    }
    double* dst = plan.partials + m * 64;
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) dst[c * 8 + ch] = acc[c][ch];
}

// Adjoint, pass 2: per active node, the sum of its corner partials in the
// plan's fixed order.
__global__ __launch_bounds__(kBlock) void k_scatter_nodes(GridPlanDev plan, int C,
                                                          const double* __restrict__ part,
                                                          float* __restrict__ out) {
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a >= plan.n_act) return;
    const int64_t R = plan.res;
    const int64_t plane = R * R * R;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t e = plan.node_start[a]; e < plan.node_start[a + 1]; ++e) {
        const int32_t src = plan.node_src[e];
        const double* pp = part + (int64_t)(src >> 3) * 64 + (src & 7) * 8;
        for (int ch = 0; ch < C; ++ch) s[ch] += pp[ch];
    }
    const int32_t node = plan.node_id[a];
    for (int ch = 0; ch < C; ++ch) out[ch * plane + node] = (float)s[ch];
}

__global__ void k_scale_by(const float* __restrict__ x, int64_t n, const double* __restrict__ f,
                           float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (float)((double)x[i] * f[0]);
}

__global__ void k_fill_zero(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

int check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

template <int TONE, bool GRAD, bool LR>
void launch_rl(dim3 grid, hipStream_t st, const float* sh, int64_t ss, int64_t n, int K,
               const SigmaTable& tab, const float* mat, int64_t ms, const float* obs, int64_t os,
               double* partials, float* grad, int64_t gs, float* Lr, int64_t ls) {
    hipLaunchKernelGGL((k_render_loss<TONE, GRAD, LR>), grid, dim3(kBlock), 0, st, sh, ss, n, K,
                       tab, mat, ms, obs, os, partials, grad, gs, Lr, ls);
}

}  // namespace

int launch_render_loss(const float* sh, int64_t ss, int64_t n, int32_t K, const float* sigma,
                       const float* mat, int64_t ms, const float* obs, int64_t os, int32_t tone,
                       double* loss, float* grad, int64_t gs, float* Lr, int64_t ls,
                       void* stream) {
    SigmaTable tab;
    for (int k = 0; k < FIPT_MAX_LEVELS; ++k) {
        tab.s[k] = k < K ? sigma[k] : 0.0f;
        tab.inv_gap[k] = (k + 1 < K) ? 1.0f / (sigma[k + 1] - sigma[k]) : 0.0f;
    }
    const int64_t want = (n + kBlock - 1) / kBlock;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, kMaxPartials));
    hipStream_t st = (hipStream_t)stream;
    double* partials = loss + 1;
    const dim3 grid(blocks);
    const bool g = grad != nullptr, l = Lr != nullptr;
#define FIPT_RL(T, G, L) launch_rl<T, G, L>(grid, st, sh, ss, n, K, tab, mat, ms, obs, os, partials, grad, gs, Lr, ls)
    if (tone == 0) {
        if (g && l) FIPT_RL(0, true, true);
        else if (g) FIPT_RL(0, true, false);
        else if (l) FIPT_RL(0, false, true);
        else FIPT_RL(0, false, false);
    } else {
        if (g && l) FIPT_RL(1, true, true);
        else if (g) FIPT_RL(1, true, false);
        else if (l) FIPT_RL(1, false, true);
        else FIPT_RL(1, false, false);
    }
#undef FIPT_RL
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
        g.scale[k] = (float)(R - 1) / (bmax[k] - bmin[k]);
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
    const int64_t total = (int64_t)C * p.res * p.res * p.res;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, st, grad_grid, total);
    int rc = check("grid_scatter fill");
    if (rc) return rc;
    if (p.n_occ == 0) return FIPT_OK;
    const unsigned cb = (unsigned)((p.n_occ + kBlock - 1) / kBlock);
    switch (C) {
#define FIPT_SC(N) case N: hipLaunchKernelGGL(k_scatter_cells<N>, dim3(cb), dim3(kBlock), 0, st, p, g, gp, gs); break
        FIPT_SC(1); FIPT_SC(2); FIPT_SC(3); FIPT_SC(4);
        FIPT_SC(5); FIPT_SC(6); FIPT_SC(7); FIPT_SC(8);
#undef FIPT_SC
        default: return fail(FIPT_EINVAL, "channels must be in [1, 8]");
    }
    rc = check("grid_scatter cells");
    if (rc) return rc;
    if (p.n_act == 0) return FIPT_OK;
    hipLaunchKernelGGL(k_scatter_nodes, dim3((unsigned)((p.n_act + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, p, C, (const double*)p.partials, grad_grid);
    return check("grid_scatter nodes");
}

}  // namespace fipt
