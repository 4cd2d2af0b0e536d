// Host set-up of the deterministic adjoint of the trilinear material grid
// (fipt_grid_plan_*) and the scatter entry point.
//
// The plan sorts the points by grid cell once and cuts every cell's run into
// segments of at most 48 points.  The adjoint then runs with no atomics:
// the per-point gradient planes are first copied into 32-byte records (so
// the cell-ordered pass reads one line per point, not one per channel);
// every segment sums weight * gradient of its points into the eight corners
// of its cell (points in index order), straight into the cell's partials
// when the cell has a single segment; every cell with several segments sums
// them (in order); and every node next to an occupied cell sums the corner
// partials of at most eight cells (in order).  The result is bitwise
// reproducible.
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
    void* ptrs[] = {p->d.perm,      p->d.seg_start, p->d.seg_cell, p->d.cell_seg,
                    p->d.node_id,   p->d.node_start, p->d.node_src, p->d.pos,
                    p->d.seg_part,  p->d.cell_part, p->d.seg_row,  p->d.multi_cell,
                    p->d.gp_rec};
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
    const int64_t cr = res - 1;
    std::vector<std::pair<int64_t, int32_t>> key(n);
    double scale[3];
    for (int k = 0; k < 3; ++k) scale[k] = (double)(res - 1) / ((double)bmax[k] - (double)bmin[k]);
    const double top = (double)(res - 1);
    for (int64_t p = 0; p < n; ++p) {
        int64_t idx[3];
        for (int k = 0; k < 3; ++k) {
            const float x = pos[k * n + p];
            if (!std::isfinite(x)) return fail(FIPT_EINVAL, "point %lld has a non-finite position", (long long)p);
            const double u = std::fmin(std::fmax(((double)x - (double)bmin[k]) * scale[k], 0.0), top);
            idx[k] = std::min<int64_t>((int64_t)std::floor(u), res - 2);
        }
        key[p] = {idx[0] + cr * (idx[1] + cr * idx[2]), (int32_t)p};
    }
    std::sort(key.begin(), key.end());
    // segments: runs of at most kSegmentMax points of one cell, so a cell
    // seen by many pixels does not serialise on one thread
    constexpr int64_t kSegmentMax = 48;
    std::vector<int32_t> perm(n), seg_start, seg_cell, cell_seg, cell_id;
    for (int64_t q = 0; q < n; ++q) {
        perm[q] = key[q].second;
        const bool new_cell = q == 0 || key[q].first != key[q - 1].first;
        if (new_cell || q - seg_start.back() >= kSegmentMax) {
            if (new_cell) {
                cell_seg.push_back((int32_t)seg_start.size());
                cell_id.push_back((int32_t)key[q].first);
            }
            seg_start.push_back((int32_t)q);
            seg_cell.push_back((int32_t)key[q].first);
        }
    }
    seg_start.push_back((int32_t)n);
    cell_seg.push_back((int32_t)seg_cell.size());
    const int64_t S = (int64_t)seg_cell.size();
    const int64_t M = (int64_t)cell_id.size();
    // a cell with one segment takes its partials straight from pass 1
    std::vector<int32_t> seg_row(S), multi_cell;
    for (int64_t m = 0; m < M; ++m) {
        const int32_t g0 = cell_seg[m], g1 = cell_seg[m + 1];
        if (g1 - g0 == 1) {
            seg_row[g0] = (int32_t)m;
        } else {
            multi_cell.push_back((int32_t)m);
            for (int32_t g = g0; g < g1; ++g) seg_row[g] = -1 - g;
        }
    }
    std::vector<std::pair<int64_t, int32_t>> nk;
    nk.reserve(8 * M);
    for (int64_t m = 0; m < M; ++m) {
        const int64_t c = cell_id[m];
        const int64_t i = c % cr, j = (c / cr) % cr, k = c / (cr * cr);
        for (int corner = 0; corner < 8; ++corner) {
            const int64_t ni = i + (corner & 1), nj = j + ((corner >> 1) & 1), nkk = k + (corner >> 2);
            nk.push_back({ni + res * (nj + (int64_t)res * nkk), (int32_t)((m << 3) | corner)});
        }
    }
    std::sort(nk.begin(), nk.end());
    std::vector<int32_t> node_id, node_start, node_src(nk.size());
    for (size_t e = 0; e < nk.size(); ++e) {
        node_src[e] = nk[e].second;
        if (e == 0 || nk[e].first != nk[e - 1].first) {
            node_start.push_back((int32_t)e);
            node_id.push_back((int32_t)nk[e].first);
        }
    }
    node_start.push_back((int32_t)nk.size());
    // positions stored in sorted order: the adjoint reads them contiguously
    std::vector<float> pcopy(3 * n);
    for (int k = 0; k < 3; ++k)
        for (int64_t q = 0; q < n; ++q) pcopy[k * n + q] = pos[k * n + perm[q]];

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
    d.n_seg = S;
    d.n_cell = M;
    d.n_multi = (int64_t)multi_cell.size();
    d.n_act = (int64_t)node_id.size();
    int rc;
    if ((rc = upload(&d.perm, perm, &p->bytes)) || (rc = upload(&d.seg_start, seg_start, &p->bytes)) ||
        (rc = upload(&d.seg_cell, seg_cell, &p->bytes)) || (rc = upload(&d.cell_seg, cell_seg, &p->bytes)) ||
        (rc = upload(&d.node_id, node_id, &p->bytes)) ||
        (rc = upload(&d.node_start, node_start, &p->bytes)) ||
        (rc = upload(&d.node_src, node_src, &p->bytes)) || (rc = upload(&d.pos, pcopy, &p->bytes)) ||
        (rc = upload(&d.seg_row, seg_row, &p->bytes)) ||
        (rc = upload(&d.multi_cell, multi_cell, &p->bytes))) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&d.seg_part), sizeof(double) * 64 * std::max<int64_t>(S, 1));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&d.cell_part), sizeof(double) * 64 * std::max<int64_t>(M, 1));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.gp_rec), sizeof(float) * 8 * n);
    if (e != hipSuccess) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(FIPT_ENOMEM, "hipMalloc partials: %s", hipGetErrorString(e));
    }
    p->bytes += (int64_t)(sizeof(double) * 64 * (S + M) + sizeof(float) * 8 * n);
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

}  // extern "C"
