// Host set-up of the deterministic adjoint of the trilinear material grid
// (fipt_grid_plan_*) and the scatter entry point.
//
// The plan sorts the points once by home brick (the node brick that holds
// the lower corner of the point's cell), cell and index, and cuts every
// cell's run into columns of at most kColumnMax points.  A brick's column
// list holds its home columns and the halo columns: those of cells in the
// lower neighbouring bricks whose upper corners are nodes of this brick.
// The adjoint runs one workgroup per brick: every thread sums one column in
// double in point order, and the column sums are added into the brick's
// nodes as 64-bit fixed-point integers whose scale the brick derives from
// its largest column sum, so the node sums do not depend on the order of
// the additions; the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "fipt_internal.hpp"

struct fipt_grid_plan_s {
    int32_t device = 0;
    fipt::GridPlanDev d;
    int64_t bytes = 0;
};

using namespace fipt;

namespace {

void plan_free(fipt_grid_plan p) {
    if (!p) return;
    void* ptrs[] = {p->d.pts, p->d.cols, p->d.units, p->d.multi, p->d.part, p->d.hcol, p->d.colq,
                    p->d.csum};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

template <typename T>
int upload(T** dst, const std::vector<T>& src, int64_t* bytes) {
    const size_t nb = sizeof(T) * std::max<size_t>(src.size(), 1);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), nb);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "hipMalloc: %s",
                    hipGetErrorString(e));
    *bytes += (int64_t)nb;
    if (!src.empty()) {
        e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(FIPT_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    return FIPT_OK;
}

}  // namespace

extern "C" {

int fipt_grid_plan_create(const float* pos, int64_t n, int32_t res, const float* bmin,
                          const float* bmax, int32_t device, fipt_grid_plan* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pos || !bmin || !bmax) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FIPT_EINVAL, "n must be in [1, 2^31)");
    if (res < 2 || res > 1024) return fail(FIPT_EINVAL, "res must be in [2, 1024]");
    for (int k = 0; k < 3; ++k)
        if (!(bmax[k] > bmin[k])) return fail(FIPT_EINVAL, "empty grid box on axis %d", k);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(FIPT_EINVAL, "device %d not available", device);
    // cell of every point, exactly as the device computes it
    const int64_t B[3] = {kBrickX, kBrickY, kBrickZ};
    int64_t nb[3];
    for (int k = 0; k < 3; ++k) nb[k] = (res + B[k] - 1) / B[k];
    double scale[3];
    for (int k = 0; k < 3; ++k) scale[k] = (double)(res - 1) / ((double)bmax[k] - (double)bmin[k]);
    const double top = (double)(res - 1);
    // key: home brick (x fastest) << 40 | cell within the brick << 31 | point
    std::vector<uint64_t> key(n);
    for (int64_t p = 0; p < n; ++p) {
        int64_t idx[3];
        for (int k = 0; k < 3; ++k) {
            const float x = pos[k * n + p];
            if (!std::isfinite(x)) return fail(FIPT_EINVAL, "point %lld has a non-finite position", (long long)p);
            const double u = std::fmin(std::fmax(((double)x - (double)bmin[k]) * scale[k], 0.0), top);
            idx[k] = std::min<int64_t>((int64_t)std::floor(u), res - 2);
        }
        const uint64_t hb = (uint64_t)(idx[0] / B[0] + nb[0] * (idx[1] / B[1] + nb[1] * (idx[2] / B[2])));
        const uint64_t lc = (uint64_t)(idx[0] % B[0] + B[0] * (idx[1] % B[1] + B[1] * (idx[2] % B[2])));
        key[p] = hb << 40 | lc << 31 | (uint64_t)p;
    }
    std::sort(key.begin(), key.end());
    // columns: runs of at most kColumnMax points of one cell; each goes to
    // its home brick and to the up to seven bricks above it whose first
    // node is the cell's upper corner on some axis
    const int64_t n_bricks = nb[0] * nb[1] * nb[2];
    struct Col {
        int64_t brick;
        int32_t start, word, home;
    };
    std::vector<Col> cols;
    cols.reserve(n / 2 + 16);
    // home column of every point in sorted order; a column never crosses a
    // multiple of 16 points, so the fused loss kernel finds each column's
    // points within one row of 16 lanes
    std::vector<int32_t> colq(n);
    int32_t n_home = 0;
    for (int64_t q = 0; q < n;) {
        const uint64_t cell_key = key[q] >> 31;
        int64_t e = q + 1;
        while (e < n && (key[e] >> 31) == cell_key) ++e;
        const int64_t hb = (int64_t)(cell_key >> 9);
        const int64_t lc = (int64_t)(cell_key & 511);
        const int64_t l[3] = {lc % B[0], (lc / B[0]) % B[1], lc / (B[0] * B[1])};
        const int64_t h[3] = {hb % nb[0], (hb / nb[0]) % nb[1], hb / (nb[0] * nb[1])};
        for (int64_t a = q; a < e;) {
            const int32_t cnt = (int32_t)std::min<int64_t>(std::min<int64_t>(kColumnMax, e - a),
                                                           16 - (a & 15));
            const int32_t home = n_home++;
            for (int64_t v = a; v < a + cnt; ++v) colq[v] = home;
            for (int t = 0; t < 8; ++t) {
                int64_t tb[3], tl[3];
                bool ok = true;
                for (int k = 0; k < 3; ++k) {
                    const int d = (t >> k) & 1;
                    // shifting to the next brick on axis k needs the cell on
                    // the brick's last layer and a brick above
                    if (d && (l[k] != B[k] - 1 || h[k] + 1 >= nb[k])) ok = false;
                    tb[k] = h[k] + d;
                    tl[k] = l[k] - d * B[k];
                }
                if (!ok) continue;
                const int64_t brick = tb[0] + nb[0] * (tb[1] + nb[1] * tb[2]);
                const int32_t word = cnt | (int32_t)(tl[0] + 1) << 5 | (int32_t)(tl[1] + 1) << 11 |
                                     (int32_t)(tl[2] + 1) << 17;
                cols.push_back({brick, (int32_t)a, word, home});
            }
            a += cnt;
        }
        q = e;
    }
    if ((int64_t)cols.size() >= (int64_t(1) << 31))
        return fail(FIPT_EINVAL, "%lld columns: too many for one plan", (long long)cols.size());
    // every brick's columns together, in cell order (halo cells first on an
    // axis), then point order
    std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) {
        if (a.brick != b.brick) return a.brick < b.brick;
        return (a.word >> 5) < (b.word >> 5);  // (lz, ly, lx), each + 1 in six bits
    });
    std::vector<int32_t> brick_col(n_bricks + 1, 0);
    for (const Col& c : cols) ++brick_col[c.brick + 1];
    for (int64_t b = 0; b < n_bricks; ++b) brick_col[b + 1] += brick_col[b];
    std::vector<int2> cword(cols.size());
    std::vector<int32_t> hcol(cols.size());
    for (size_t c = 0; c < cols.size(); ++c) {
        cword[c] = make_int2(cols[c].start, cols[c].word);
        hcol[c] = cols[c].home;
    }
    // work units: every brick's columns in runs of at most `per` (a brick
    // with no columns is one empty unit, which writes zeros)
    auto make_units = [&](int32_t per, std::vector<int4>& units, std::vector<int4>& multi) {
        int32_t slots = 0;
        for (int64_t b = 0; b < n_bricks; ++b) {
            const int32_t c0 = brick_col[b], c1 = brick_col[b + 1];
            const int32_t nu = std::max<int32_t>(1, (c1 - c0 + per - 1) / per);
            if (nu == 1) {
                units.push_back(make_int4((int32_t)b, c0, c1, -1));
                continue;
            }
            multi.push_back(make_int4((int32_t)b, slots, nu, 0));
            for (int32_t u = 0; u < nu; ++u)
                units.push_back(make_int4((int32_t)b, c0 + u * per,
                                          std::min<int32_t>(c1, c0 + (u + 1) * per), slots + u));
            slots += nu;
        }
        // heaviest units first: the hardware deals workgroups to the XCDs in
        // turn, and the long units start early instead of forming the tail
        std::stable_sort(units.begin(), units.end(),
                         [](const int4& a, const int4& b) { return a.z - a.y > b.z - b.y; });
        return slots;
    };
    std::vector<int4> units, multi;
    const int32_t slots = make_units(kAdjUnit, units, multi);
    // points in sorted order: (x, y, z, index)
    std::vector<float4> pts(n);
    for (int64_t q = 0; q < n; ++q) {
        const int64_t p = (int64_t)(key[q] & 0x7fffffffu);
        int32_t pi = (int32_t)p;
        float w;
        std::memcpy(&w, &pi, 4);
        pts[q] = make_float4(pos[p], pos[n + p], pos[2 * n + p], w);
    }

    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(FIPT_EHIP, "hipSetDevice(%d) failed", device);
    fipt_grid_plan p = new fipt_grid_plan_s();
    p->device = device;
    GridPlanDev& d = p->d;
    std::memset(&d, 0, sizeof(d));
    d.res = res;
    d.n_points = n;
    for (int k = 0; k < 3; ++k) {
        d.bmin[k] = bmin[k];
        d.bmax[k] = bmax[k];
    }
    for (int k = 0; k < 3; ++k) d.nb[k] = (int32_t)nb[k];
    d.n_bricks = n_bricks;
    d.n_cols = (int64_t)cols.size();
    d.n_units = (int64_t)units.size();
    d.n_multi = (int64_t)multi.size();
    d.n_slots = slots;
    d.n_home = n_home;
    int rc;
    if ((rc = upload(&d.pts, pts, &p->bytes)) || (rc = upload(&d.cols, cword, &p->bytes)) ||
        (rc = upload(&d.units, units, &p->bytes)) || (rc = upload(&d.multi, multi, &p->bytes)) ||
        (rc = upload(&d.hcol, hcol, &p->bytes)) || (rc = upload(&d.colq, colq, &p->bytes))) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    }
    const size_t part_bytes = sizeof(double) * 8 * kBrickNodes * std::max<int64_t>(slots, 1);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&d.part), part_bytes);
    if (e != hipSuccess) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(FIPT_ENOMEM, "hipMalloc unit sums: %s", hipGetErrorString(e));
    }
    p->bytes += (int64_t)part_bytes;
    const size_t cs_bytes = sizeof(float) * 40 * (size_t)std::max<int32_t>(n_home, 1);
    e = hipMalloc(reinterpret_cast<void**>(&d.csum), cs_bytes);
    if (e != hipSuccess) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(FIPT_ENOMEM, "hipMalloc column sums: %s", hipGetErrorString(e));
    }
    p->bytes += (int64_t)cs_bytes;
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = p;
    return FIPT_OK;
}

int fipt_grid_plan_destroy(fipt_grid_plan p) {
    clear_error();
    if (!p) return FIPT_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    plan_free(p);
    if (prev >= 0) (void)hipSetDevice(prev);
    return FIPT_OK;
}

int fipt_grid_scatter(fipt_grid_plan p, const float* grad_points, int32_t channels,
                      int64_t gp_stride, float* grad_grid, void* stream) {
    clear_error();
    if (!p || !grad_points || !grad_grid) return fail(FIPT_EINVAL, "NULL argument");
    if (channels < 1 || channels > 8) return fail(FIPT_EINVAL, "channels must be in [1, 8]");
    if (gp_stride < p->d.n_points) return fail(FIPT_EINVAL, "gp_stride < plan point count");
    return launch_grid_scatter(p->d, grad_points, channels, gp_stride, grad_grid, stream);
}

int fipt_grid_plan_order(fipt_grid_plan p, int32_t* order_host) {
    clear_error();
    if (!p || !order_host) return fail(FIPT_EINVAL, "NULL argument");
    std::vector<float4> pts(p->d.n_points);
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(p->device) != hipSuccess) return fail(FIPT_EHIP, "hipSetDevice(%d) failed", p->device);
    const hipError_t e = hipMemcpy(pts.data(), p->d.pts, sizeof(float4) * pts.size(), hipMemcpyDeviceToHost);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail(FIPT_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    for (size_t q = 0; q < pts.size(); ++q) std::memcpy(order_host + q, &pts[q].w, 4);
    return FIPT_OK;
}

int fipt_grid_plan_permute(fipt_grid_plan p, const float* src, int32_t planes, int64_t src_stride,
                           float* dst, int64_t dst_stride, void* stream) {
    clear_error();
    if (!p || !src || !dst) return fail(FIPT_EINVAL, "NULL argument");
    if (planes < 1) return fail(FIPT_EINVAL, "planes must be >= 1");
    if (src_stride < p->d.n_points || dst_stride < p->d.n_points)
        return fail(FIPT_EINVAL, "a stride is smaller than the plan's point count");
    const char* s0 = reinterpret_cast<const char*>(src);
    const char* d0 = reinterpret_cast<const char*>(dst);
    const int64_t span_s = 4 * ((planes - 1) * src_stride + p->d.n_points);
    const int64_t span_d = 4 * ((planes - 1) * dst_stride + p->d.n_points);
    if (s0 < d0 + span_d && d0 < s0 + span_s) return fail(FIPT_EINVAL, "src and dst overlap");
    return launch_plan_permute(p->d, src, planes, src_stride, dst, dst_stride, stream);
}

int fipt_grid_render_loss(fipt_grid_plan p, const float* grid, const fipt_shading* sh,
                          int32_t n_levels, const float* sigma_host, const float* observed,
                          int64_t obs_stride, int32_t tonemap, double* loss_dev, float* grad_grid,
                          float* grad_points, int64_t gp_stride, void* stream) {
    clear_error();
    if (!p || !grid || !sh || !sh->planes || !sigma_host || !observed || !loss_dev || !grad_grid)
        return fail(FIPT_EINVAL, "NULL argument");
    const int64_t n = p->d.n_points;
    if (n_levels < 2 || n_levels > FIPT_MAX_LEVELS)
        return fail(FIPT_EINVAL, "n_levels must be in [2, %d], got %d", FIPT_MAX_LEVELS, n_levels);
    for (int k = 0; k < n_levels; ++k) {
        if (!std::isfinite(sigma_host[k])) return fail(FIPT_EINVAL, "sigma[%d] is not finite", k);
        if (k > 0 && !(sigma_host[k] > sigma_host[k - 1]))
            return fail(FIPT_EINVAL, "sigma must be strictly increasing");
    }
    if (sh->stride < n || obs_stride < n) return fail(FIPT_EINVAL, "a stride is smaller than n");
    if (grad_points && gp_stride < n) return fail(FIPT_EINVAL, "gp_stride < n");
    if (tonemap != FIPT_TONEMAP_NONE && tonemap != FIPT_TONEMAP_LOG_SRGB)
        return fail(FIPT_EINVAL, "unknown tonemap %d", tonemap);
    return launch_grid_render_loss(p->d, grid, sh->planes, sh->stride, n_levels, sigma_host,
                                   observed, obs_stride, tonemap, loss_dev, loss_dev + 1,
                                   grad_points, gp_stride, grad_grid, stream);
}

}  // extern "C"
