// The voxel radiance cache of Sec. 4.2 for gfx950: average pooling of the
// observed pixels onto a grid over the scene (the L' that the query of Eq. 9
// reads), and the conversion of a grid into the scene's sparse form.
//
// The pixel-to-voxel map is fixed by the cameras, so a plan sorts the pixels
// by voxel once (host counting sort, pixels of a voxel in index order) and
// keeps a dense start array over all voxels.  The pooling kernel then runs
// one thread per voxel over the whole grid: it sums its pixels' observations
// in double, in pixel order, and writes the mean, or zero for an empty voxel,
// so every voxel is written in one coalesced pass and the result does not
// depend on scheduling.  The grid is ~4 (R^3 + n) bytes of plan and
// 12 R^3 bytes of output: 268 MB in all at R = 256 for a million pixels,
// which HBM holds with room to spare.
//
// The bake reads the grid at random surface points, so the scene keeps it
// sparse: pixels only ever land on surfaces, and of the 16.8 M voxels of a
// 256^3 grid over a room a few per cent are occupied.  One 16-byte word per
// brick of 4 x 4 x 4 voxels (occupancy bits and the number of occupied
// voxels in earlier bricks) and the occupied values in brick order take
// ~9 MB instead of 268 MB, and hits close together on a surface read the
// same words and value lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fipt_internal.hpp"

struct fipt_voxel_plan_s {
    int32_t device = 0;
    int64_t n = 0;           // pixels
    int32_t res = 0;
    int64_t n_vox = 0;       // res^3
    int32_t* start = nullptr;  // [n_vox + 1] ranges into order
    int32_t* order = nullptr;  // [n] pixels grouped by voxel, index order within one
    int64_t bytes = 0;
};

namespace fipt {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_voxel_pool(const int32_t* __restrict__ start,
                                                       const int32_t* __restrict__ order,
                                                       int64_t n_vox,
                                                       const float* __restrict__ obs, int64_t os,
                                                       float* __restrict__ out, int64_t cs) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n_vox; v += step) {
        const int32_t s = start[v], e = start[v + 1];
        double r = 0.0, g = 0.0, b = 0.0;
        int32_t i = s;
        // four pixels' loads in flight at once; the additions keep pixel order
        for (; i + 4 <= e; i += 4) {
            int64_t p[4];
            float q[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] = order[i + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                q[u][0] = obs[p[u]];
                q[u][1] = obs[os + p[u]];
                q[u][2] = obs[2 * os + p[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                r += q[u][0];
                g += q[u][1];
                b += q[u][2];
            }
        }
        for (; i < e; ++i) {
            const int64_t p = order[i];
            r += obs[p];
            g += obs[os + p];
            b += obs[2 * os + p];
        }
        const int32_t k = e - s;
        float mr = 0.0f, mg = 0.0f, mb = 0.0f;
        if (k > 0) {
            mr = (float)(r / (double)k);
            mg = (float)(g / (double)k);
            mb = (float)(b / (double)k);
        }
        out[v] = mr;
        out[cs + v] = mg;
        out[2 * cs + v] = mb;
    }
}

// Voxel of lane `lane` of brick `w` (B bricks per axis): lane bits
// (k % 4, j % 4, i % 4) from high to low.
__device__ __forceinline__ void brick_voxel(int64_t w, int lane, int32_t nb, int32_t& i,
                                            int32_t& j, int32_t& k) {
    const int32_t bx = (int32_t)(w % nb), by = (int32_t)((w / nb) % nb), bz = (int32_t)(w / ((int64_t)nb * nb));
    i = 4 * bx + (lane & 3);
    j = 4 * by + ((lane >> 2) & 3);
    k = 4 * bz + (lane >> 4);
}

// Occupancy of an R^3 grid given as planes [3][cs], one wavefront per brick
// of 4 x 4 x 4 voxels (one word): a voxel is occupied when any channel is
// non-zero; .z holds the brick's occupied count until the scan turns it
// into a rank.
__global__ __launch_bounds__(kBlock) void k_voxel_words(uint4* __restrict__ words,
                                                        const float* __restrict__ cache,
                                                        int64_t cs, int32_t res) {
    const int lane = threadIdx.x & 63;
    const int32_t nb = (res + 3) / 4;
    const int64_t n_words = (int64_t)nb * nb * nb;
    const int64_t wave0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t step = ((int64_t)gridDim.x * kBlock) >> 6;
    for (int64_t w = wave0; w < n_words; w += step) {
        int32_t i, j, k;
        brick_voxel(w, lane, nb, i, j, k);
        bool occ = false;
        if (i < res && j < res && k < res) {
            const int64_t v = ((int64_t)k * res + j) * res + i;
            occ = (cache[v] != 0.0f) | (cache[cs + v] != 0.0f) | (cache[2 * cs + v] != 0.0f);
        }
        const uint64_t m = __builtin_amdgcn_ballot_w64(occ);
        if (lane == 0)
            words[w] = make_uint4((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)__popcll(m), 0u);
    }
}

// Exclusive scan of the words' counts (.z) into ranks, in three passes over
// tiles of 1024 words: each tile scanned by one workgroup (its total kept),
// the tile totals scanned by one workgroup (the grand total to *total), the
// tile offsets added.
constexpr int kScanTile = (int)kVoxelScanTile;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* lds, uint32_t& sum) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t incl = x;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t up = __shfl_up(incl, d, 64);
        if (lane >= d) incl += up;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int w = 0; w < kScanTile / 64; ++w) {
            const uint32_t v = lds[w];
            lds[w] = run;
            run += v;
        }
        lds[kScanTile / 64] = run;
    }
    __syncthreads();
    sum = lds[kScanTile / 64];
    const uint32_t r = lds[wave] + incl - x;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanTile) void k_voxel_scan_tiles(uint4* __restrict__ words,
                                                                int64_t n_words,
                                                                uint32_t* __restrict__ tile_sum) {
    __shared__ uint32_t lds[kScanTile / 64 + 1];
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    const uint32_t x = i < n_words ? words[i].z : 0u;
    uint32_t sum;
    const uint32_t r = block_exclusive_scan(x, lds, sum);
    if (i < n_words) words[i].z = r;
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kScanTile) void k_voxel_scan_totals(uint32_t* __restrict__ tile_sum,
                                                                 int64_t n_tiles,
                                                                 int64_t* __restrict__ total) {
    __shared__ uint32_t lds[kScanTile / 64 + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += kScanTile) {
        const int64_t i = base + threadIdx.x;
        const uint32_t x = i < n_tiles ? tile_sum[i] : 0u;
        uint32_t sum;
        const uint32_t r = block_exclusive_scan(x, lds, sum);
        if (i < n_tiles) tile_sum[i] = carry + r;
        carry += sum;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanTile) void k_voxel_scan_add(uint4* __restrict__ words,
                                                              int64_t n_words,
                                                              const uint32_t* __restrict__ tile_sum) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    if (i < n_words) words[i].z += tile_sum[blockIdx.x];
}

// Occupied voxels' values in brick order, one wavefront per brick.
__global__ __launch_bounds__(kBlock) void k_voxel_compact(float4* __restrict__ dst,
                                                          const uint4* __restrict__ words,
                                                          const float* __restrict__ cache,
                                                          int64_t cs, int32_t res) {
    const int lane = threadIdx.x & 63;
    const int32_t nb = (res + 3) / 4;
    const int64_t n_words = (int64_t)nb * nb * nb;
    const int64_t wave0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t step = ((int64_t)gridDim.x * kBlock) >> 6;
    for (int64_t w = wave0; w < n_words; w += step) {
        const uint4 wd = words[w];
        const uint64_t m = ((uint64_t)wd.y << 32) | wd.x;
        if ((m >> lane) & 1ull) {
            int32_t i, j, k;
            brick_voxel(w, lane, nb, i, j, k);
            const int64_t v = ((int64_t)k * res + j) * res + i;
            const uint32_t idx = wd.z + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            dst[idx] = make_float4(cache[v], cache[cs + v], cache[2 * cs + v], 0.0f);
        }
    }
}

int grid_for(int64_t n) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)cus * 32));
}

int check_voxel(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

}  // namespace

int launch_voxel_words(uint4* words, const float* cache, int64_t stride, int32_t res,
                       uint32_t* tile_sum, int64_t* total, void* stream) {
    const int64_t nb = (res + 3) / 4;
    const int64_t n_words = nb * nb * nb;
    const int64_t n_tiles = (n_words + kScanTile - 1) / kScanTile;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_voxel_words, dim3(grid_for(n_words * 64)), dim3(kBlock), 0, st, words,
                       cache, stride, res);
    int rc = check_voxel("voxel_words");
    if (rc) return rc;
    hipLaunchKernelGGL(k_voxel_scan_tiles, dim3((unsigned)n_tiles), dim3(kScanTile), 0, st, words,
                       n_words, tile_sum);
    rc = check_voxel("voxel_scan_tiles");
    if (rc) return rc;
    hipLaunchKernelGGL(k_voxel_scan_totals, dim3(1), dim3(kScanTile), 0, st, tile_sum, n_tiles, total);
    rc = check_voxel("voxel_scan_totals");
    if (rc) return rc;
    hipLaunchKernelGGL(k_voxel_scan_add, dim3((unsigned)n_tiles), dim3(kScanTile), 0, st, words,
                       n_words, tile_sum);
    return check_voxel("voxel_scan_add");
}

int launch_voxel_compact(float4* dst, const uint4* words, const float* cache, int64_t stride,
                         int32_t res, void* stream) {
    const int64_t nb = (res + 3) / 4;
    hipLaunchKernelGGL(k_voxel_compact, dim3(grid_for(nb * nb * nb * 64)), dim3(kBlock), 0,
                       (hipStream_t)stream, dst, words, cache, stride, res);
    return check_voxel("voxel_compact");
}

}  // namespace fipt

using namespace fipt;

extern "C" {

int fipt_voxel_plan_create(const float* pos_host, int64_t n, int32_t res, const float* bmin_host,
                           const float* bmax_host, int32_t device, fipt_voxel_plan* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pos_host || !bmin_host || !bmax_host) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FIPT_EINVAL, "n must be in [1, 2^31)");
    if (res < 1 || res > kMaxVoxelRes)
        return fail(FIPT_EINVAL, "res must be in [1, %d], got %d", kMaxVoxelRes, res);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(bmin_host[a]) || !std::isfinite(bmax_host[a]) ||
            !(bmax_host[a] > bmin_host[a]))
            return fail(FIPT_EINVAL, "the box must be finite with bmin < bmax on every axis");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(FIPT_EINVAL, "device %d not available", device);
    const int64_t n_vox = (int64_t)res * res * res;
    // voxel of every pixel (double arithmetic on the float inputs), then a
    // stable counting sort
    std::vector<int32_t> vox(n);
    for (int64_t p = 0; p < n; ++p) {
        int64_t ijk[3];
        for (int a = 0; a < 3; ++a) {
            const double lo = bmin_host[a], hi = bmax_host[a];
            const double u = ((double)pos_host[a * n + p] - lo) * res / (hi - lo);
            double f = std::floor(u);
            if (!(f >= 0.0)) f = 0.0;   // also NaN
            if (f > res - 1) f = res - 1;
            ijk[a] = (int64_t)f;
        }
        vox[p] = (int32_t)((ijk[2] * res + ijk[1]) * res + ijk[0]);
    }
    std::vector<int32_t> start(n_vox + 1, 0);
    for (int64_t p = 0; p < n; ++p) ++start[vox[p] + 1];
    for (int64_t v = 0; v < n_vox; ++v) start[v + 1] += start[v];
    std::vector<int32_t> order(n);
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t p = 0; p < n; ++p) order[fill[vox[p]]++] = (int32_t)p;
    }

    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(FIPT_EHIP, "hipSetDevice(%d) failed", device);
    fipt_voxel_plan pl = new fipt_voxel_plan_s();
    pl->device = device;
    pl->n = n;
    pl->res = res;
    pl->n_vox = n_vox;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&pl->start), sizeof(int32_t) * start.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pl->order), sizeof(int32_t) * order.size());
    if (e == hipSuccess)
        e = hipMemcpy(pl->start, start.data(), sizeof(int32_t) * start.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pl->order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (pl->start) (void)hipFree(pl->start);
        if (pl->order) (void)hipFree(pl->order);
        delete pl;
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(e == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "voxel plan upload: %s",
                    hipGetErrorString(e));
    }
    pl->bytes = (int64_t)(sizeof(int32_t) * (start.size() + order.size()));
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = pl;
    return FIPT_OK;
}

int fipt_voxel_plan_destroy(fipt_voxel_plan pl) {
    clear_error();
    if (!pl) return FIPT_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(pl->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(pl->start);
    (void)hipFree(pl->order);
    delete pl;
    if (prev >= 0) (void)hipSetDevice(prev);
    return FIPT_OK;
}

int fipt_voxel_pool(fipt_voxel_plan pl, const float* observed, int64_t obs_stride, float* cache,
                    int64_t cache_stride, void* stream) {
    clear_error();
    if (!pl || !observed || !cache) return fail(FIPT_EINVAL, "NULL argument");
    if (obs_stride < pl->n) return fail(FIPT_EINVAL, "obs_stride < the plan's pixel count");
    if (cache_stride < pl->n_vox) return fail(FIPT_EINVAL, "cache_stride < res^3");
    hipLaunchKernelGGL(k_voxel_pool, dim3(grid_for(pl->n_vox)), dim3(kBlock), 0,
                       (hipStream_t)stream, pl->start, pl->order, pl->n_vox, observed, obs_stride,
                       cache, cache_stride);
    return check_voxel("voxel_pool");
}

}  // extern "C"
