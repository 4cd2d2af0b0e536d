// Host set-up of the deterministic adjoint of the trilinear material grid
// (fipt_grid_plan_*) and the scatter entry point.
//
// The plan sorts the points by grid cell once and cuts every cell's run into
// segments of at most 48 points.  The adjoint then runs with no atomics:
// the per-point gradient planes are first copied into 32-byte records (so
// the cell-ordered pass reads one line per point, not one per channel);
// every segment sums weight * gradient of its points into the eight corners
// of its cell (points in index order); and every grid node sums, for each
// occupied cell it is a corner of (in cell order), that cell's segment
// partials (in order), writing zero where no cell contributes.  The plan
// lists each node's contributions as (segment, corner) pairs, and a node
// finds its list through a bit mask of the active nodes with a prefix count
// per 64 nodes.  The result is bitwise reproducible.
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
    void* ptrs[] = {p->d.perm,       p->d.seg_start, p->d.seg_cell, p->d.cell_seg,
                    p->d.node_mask,  p->d.node_rank, p->d.node_start, p->d.node_src,
                    p->d.pos,        p->d.seg_part,  p->d.gp_rec};
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
    // node lists index their entries with 32 bits: eight per segment, each
    // entry holding the segment index and the corner in 32 bits
    if (8 * S >= (int64_t(1) << 31))
        return fail(FIPT_EINVAL, "%lld segments: too many for one plan", (long long)S);
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
    const int64_t n_nodes = (int64_t)res * res * res;
    const int64_t n_words = (n_nodes + 63) / 64;
    std::vector<uint64_t> node_mask(n_words, 0);
    // each node's list: for every occupied cell it is a corner of (cell
    // order), that cell's segments (segment order), as (segment << 3) | corner
    std::vector<int32_t> node_rank(n_words, 0), node_start, node_src;
    node_src.reserve(8 * S);
    for (size_t e = 0; e < nk.size(); ++e) {
        if (e == 0 || nk[e].first != nk[e - 1].first) {
            node_start.push_back((int32_t)node_src.size());
            node_mask[nk[e].first >> 6] |= uint64_t(1) << (nk[e].first & 63);
        }
        const int32_t m = nk[e].second >> 3, corner = nk[e].second & 7;
        for (int32_t g = cell_seg[m]; g < cell_seg[m + 1]; ++g) node_src.push_back((g << 3) | corner);
    }
    node_start.push_back((int32_t)node_src.size());
    for (int64_t w = 1; w < n_words; ++w)
        node_rank[w] = node_rank[w - 1] + __builtin_popcountll(node_mask[w - 1]);
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
    d.n_act = (int64_t)node_start.size() - 1;
    int rc;
    if ((rc = upload(&d.perm, perm, &p->bytes)) || (rc = upload(&d.seg_start, seg_start, &p->bytes)) ||
        (rc = upload(&d.seg_cell, seg_cell, &p->bytes)) || (rc = upload(&d.cell_seg, cell_seg, &p->bytes)) ||
        (rc = upload(&d.node_mask, node_mask, &p->bytes)) ||
        (rc = upload(&d.node_rank, node_rank, &p->bytes)) ||
        (rc = upload(&d.node_start, node_start, &p->bytes)) ||
        (rc = upload(&d.node_src, node_src, &p->bytes)) || (rc = upload(&d.pos, pcopy, &p->bytes))) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&d.seg_part), sizeof(double) * 64 * std::max<int64_t>(S, 1));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.gp_rec), sizeof(float) * 8 * n);
    if (e != hipSuccess) {
        plan_free(p);
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(FIPT_ENOMEM, "hipMalloc partials: %s", hipGetErrorString(e));
    }
    p->bytes += (int64_t)(sizeof(double) * 64 * S + sizeof(float) * 8 * n);
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
