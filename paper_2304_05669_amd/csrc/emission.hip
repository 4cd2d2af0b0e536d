// Per-triangle emission re-estimation (Sec. 4.4, Eq. 13) for gfx950.
//
// With the paper's assumption that an emitter reflects no light, the
// minimiser of Eq. 13 for a triangle classified as an emitter is, per colour
// channel, the median of the observed values of the pixels whose primary hit
// is that triangle; for an even count the lower of the two middle values is
// taken, so the result is one of the observations and is reproduced bit for
// bit.  Triangles that are not emitters, or that no pixel sees, get zero.
//
// The pixel-to-triangle map is fixed by the cameras, so a plan groups the
// pixels by triangle once (host counting sort, pixels of a triangle in
// index order).  A first kernel runs one wavefront per block of 64
// triangles: each lane writes zeros for its triangle unless it is an
// emitter, and the wave appends the block's emitters to a list (one atomic
// per wave).  Emitters come in runs of consecutive triangles (a lamp's
// faces), so the second kernel spreads the work by (emitter, channel) pair,
// one wavefront each, instead of leaving a block's emitters to one wave.
// A segment of at most 64 pixels is ranked directly (each lane
// counts the values below its own, ties broken by position); a longer one
// is searched by an exact radix selection over order-preserving 32-bit
// keys, eight bits per pass, with a 256-bin histogram in LDS.  Integer
// counts only, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fipt_internal.hpp"

struct fipt_emission_plan_s {
    int32_t device = 0;
    int64_t n = 0;          // pixels
    int64_t n_tris = 0;
    int32_t* order = nullptr;     // [n_seen] pixels grouped by triangle, index order within one
    int32_t* seg_start = nullptr; // [n_tris + 1] ranges into order
    int32_t* emitters = nullptr;  // [n_tris + 1]: the call's emitter list, its length last
    int64_t bytes = 0;
};

namespace fipt {
namespace {

constexpr int kWave = 64;

// Order-preserving key of a float (negative zero folded into positive zero,
// so equal values have equal keys), and its inverse.
__device__ __forceinline__ uint32_t float_key(float v) {
    uint32_t u = __float_as_uint(v == 0.0f ? 0.0f : v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Median (lower middle) of observed[c][order[s0 .. s0 + k)] for one channel,
// k >= 1, computed by the whole wave; every lane returns it.
__device__ float segment_median(const float* __restrict__ obs, const int32_t* __restrict__ order,
                                int32_t s0, int32_t k, int lane, int32_t* hist, int32_t* pick) {
    const int32_t r = (k - 1) / 2;
    if (k <= kWave) {
        const float v = lane < k ? obs[order[s0 + lane]] : 0.0f;
        int32_t below = 0;
        for (int32_t i = 0; i < k; ++i) {
            const float vi = __shfl(v, i, kWave);
            below += (vi < v) | ((vi == v) & (i < lane));
        }
        // exactly one lane < k has rank r
        const uint64_t m = __builtin_amdgcn_ballot_w64(lane < k && below == r);
        return __shfl(v, __ffsll((unsigned long long)m) - 1, kWave);
    }
    uint32_t prefix = 0, mask = 0;
    int32_t rank = r;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = lane; b < 256; b += kWave) hist[b] = 0;
        __syncthreads();
        for (int32_t i = lane; i < k; i += kWave) {
            const uint32_t key = float_key(obs[order[s0 + i]]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1);
        }
        __syncthreads();
        // lane j holds bins 4j .. 4j + 3; an inclusive scan over lanes finds
        // the bin in which the rank-th candidate falls
        const int32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                      h3 = hist[4 * lane + 3];
        const int32_t own = h0 + h1 + h2 + h3;
        int32_t incl = own;
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t up = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += up;
        }
        const int32_t excl = incl - own;
        if (rank >= excl && rank < incl) {
            int32_t rr = rank - excl, bin = 4 * lane;
            if (rr >= h0) { rr -= h0; ++bin;
                if (rr >= h1) { rr -= h1; ++bin;
                    if (rr >= h2) { rr -= h2; ++bin; } } }
            pick[0] = bin;
            pick[1] = rr;
        }
        __syncthreads();
        prefix |= (uint32_t)pick[0] << shift;
        mask |= 255u << shift;
        rank = pick[1];
        __syncthreads();
    }
    return key_float(prefix);
}

// Zero the non-emitters' outputs and list the emitters (list length in
// list[n_tris], zeroed beforehand).  The list's order depends on
// scheduling; each emitter's result does not.
__global__ __launch_bounds__(kWave) void k_emission_list(const uint8_t* __restrict__ emitter,
                                                          int64_t n_tris, float* __restrict__ le,
                                                          int64_t ls, int32_t* __restrict__ list) {
    const int lane = threadIdx.x;
    for (int64_t b0 = (int64_t)blockIdx.x * kWave; b0 < n_tris; b0 += (int64_t)gridDim.x * kWave) {
        const int64_t t = b0 + lane;
        const bool em = t < n_tris && emitter[t] != 0;
        if (t < n_tris && !em) {
            le[t] = 0.0f;
            le[ls + t] = 0.0f;
            le[2 * ls + t] = 0.0f;
        }
        const uint64_t m = __builtin_amdgcn_ballot_w64(em);
        if (m == 0) continue;
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(list + n_tris, (int32_t)__popcll(m));
        base = __shfl(base, 0, kWave);
        if (em) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)t;
    }
}

// One wavefront per (emitter, channel) pair of the list.
__global__ __launch_bounds__(kWave) void k_emission_median(
    const int32_t* __restrict__ order, const int32_t* __restrict__ seg_start, int64_t n_tris,
    const float* __restrict__ obs, int64_t os, const int32_t* __restrict__ list,
    float* __restrict__ le, int64_t ls) {
    __shared__ int32_t hist[256];
    __shared__ int32_t pick[2];
    const int lane = threadIdx.x;
    const int64_t items = 3 * (int64_t)list[n_tris];
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t tt = list[it / 3];
        const int c = (int)(it % 3);
        const int32_t s0 = seg_start[tt], k = seg_start[tt + 1] - s0;
        const float m = k > 0 ? segment_median(obs + c * os, order, s0, k, lane, hist, pick) : 0.0f;
        if (lane == 0) le[c * ls + tt] = m;
    }
}

__global__ void k_emission_zero_count(int32_t* count) {
    if (threadIdx.x == 0) *count = 0;
}

int check_emission(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

}  // namespace
}  // namespace fipt

using namespace fipt;

extern "C" {

int fipt_emission_plan_create(const int32_t* tri_host, int64_t n, int64_t n_tris, int32_t device,
                              fipt_emission_plan* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tri_host) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FIPT_EINVAL, "n must be in [1, 2^31)");
    if (n_tris < 1 || n_tris >= (int64_t(1) << 31))
        return fail(FIPT_EINVAL, "n_tris must be in [1, 2^31)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(FIPT_EINVAL, "device %d not available", device);
    // counting sort of the pixels by triangle (index order within one)
    std::vector<int32_t> seg(n_tris + 1, 0);
    for (int64_t p = 0; p < n; ++p) {
        const int32_t t = tri_host[p];
        if (t < -1 || t >= n_tris)
            return fail(FIPT_EINVAL, "pixel %lld names triangle %d outside [-1, %lld)", (long long)p, t,
                        (long long)n_tris);
        if (t >= 0) ++seg[t + 1];
    }
    for (int64_t t = 0; t < n_tris; ++t) seg[t + 1] += seg[t];
    std::vector<int32_t> order(std::max<int32_t>(seg[n_tris], 1));
    std::vector<int32_t> fill(seg.begin(), seg.end() - 1);
    for (int64_t p = 0; p < n; ++p)
        if (tri_host[p] >= 0) order[fill[tri_host[p]]++] = (int32_t)p;

    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(FIPT_EHIP, "hipSetDevice(%d) failed", device);
    fipt_emission_plan p = new fipt_emission_plan_s();
    p->device = device;
    p->n = n;
    p->n_tris = n_tris;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->order), sizeof(int32_t) * order.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->seg_start), sizeof(int32_t) * seg.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->emitters), sizeof(int32_t) * (n_tris + 1));
    if (e == hipSuccess)
        e = hipMemcpy(p->order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->seg_start, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->order) (void)hipFree(p->order);
        if (p->seg_start) (void)hipFree(p->seg_start);
        if (p->emitters) (void)hipFree(p->emitters);
        delete p;
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(e == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "emission plan upload: %s",
                    hipGetErrorString(e));
    }
    p->bytes = (int64_t)(sizeof(int32_t) * (order.size() + seg.size() + n_tris + 1));
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = p;
    return FIPT_OK;
}

int fipt_emission_plan_destroy(fipt_emission_plan p) {
    clear_error();
    if (!p) return FIPT_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->order);
    (void)hipFree(p->seg_start);
    (void)hipFree(p->emitters);
    delete p;
    if (prev >= 0) (void)hipSetDevice(prev);
    return FIPT_OK;
}

int fipt_emission_median(fipt_emission_plan p, const float* observed, int64_t obs_stride,
                         const uint8_t* emitter, float* le, int64_t le_stride, void* stream) {
    clear_error();
    if (!p || !observed || !emitter || !le) return fail(FIPT_EINVAL, "NULL argument");
    if (obs_stride < p->n) return fail(FIPT_EINVAL, "obs_stride < the plan's pixel count");
    if (le_stride < p->n_tris) return fail(FIPT_EINVAL, "le_stride < the plan's triangle count");
    const int64_t blocks_needed = (p->n_tris + kWave - 1) / kWave;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t waves = (int64_t)cus * 16;
    hipStream_t st = (hipStream_t)stream;
    // the list length is cleared by a kernel, not a memset node, so a caller
    // may capture the call
    hipLaunchKernelGGL(k_emission_zero_count, dim3(1), dim3(kWave), 0, st, p->emitters + p->n_tris);
    int rc = check_emission("emission_zero_count");
    if (rc) return rc;
    hipLaunchKernelGGL(k_emission_list, dim3((unsigned)std::max<int64_t>(1, std::min(blocks_needed, waves))),
                       dim3(kWave), 0, st, emitter, p->n_tris, le, le_stride, p->emitters);
    rc = check_emission("emission_list");
    if (rc) return rc;
    // at most 3 n_tris items; the kernel reads the actual count
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(3 * p->n_tris, waves));
    hipLaunchKernelGGL(k_emission_median, dim3((unsigned)grid), dim3(kWave), 0, st, p->order,
                       p->seg_start, p->n_tris, observed, obs_stride, p->emitters, le, le_stride);
    return check_emission("emission_median");
}

}  // extern "C"
