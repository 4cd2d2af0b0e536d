// Streaming bandwidth probe for gfx950: copy (c = a) and triad
// (c = a + s b) over float arrays.  It measures the HBM bandwidth a kernel
// can actually reach on the device, the denominator against which the
// memory-bound kernels of the hot path are compared besides the published
// peak.
//
// Each thread moves kUnroll 16-byte vectors per iteration of a grid-stride
// loop, all loads issued before the stores, so a wavefront keeps 4 KB of
// reads in flight; the grid is a fixed number of workgroups per CU, spread
// over all XCDs.  Stores are non-temporal: the written data is not read
// again, so it need not displace anything in L2 or the MALL.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fipt_internal.hpp"

namespace fipt {
namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;
constexpr int kBlocksPerCu = 8;

typedef float f4 __attribute__((ext_vector_type(4)));

template <bool TRIAD>
__global__ __launch_bounds__(kBlock) void k_stream(const f4* __restrict__ a, const f4* __restrict__ b,
                                                   f4* __restrict__ c, int64_t n4, float s) {
    const int64_t stride = (int64_t)gridDim.x * kBlock * kUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < n4;
         base += stride) {
        f4 va[kUnroll], vb[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kBlock;
            if (i < n4) {
                va[u] = a[i];
                if (TRIAD) vb[u] = b[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kBlock;
            if (i < n4) {
                const f4 v = TRIAD ? va[u] + s * vb[u] : va[u];
                __builtin_nontemporal_store(v, c + i);
            }
        }
    }
}

// Tail of fewer than four floats (n not a multiple of 4).
__global__ void k_stream_tail(const float* a, const float* b, float* c, int64_t from, int64_t n,
                              float s, int triad) {
    const int64_t i = from + threadIdx.x;
    if (i < n) c[i] = triad ? a[i] + s * b[i] : a[i];
}

}  // namespace

int launch_stream(int32_t kind, const float* a, const float* b, float* c, int64_t n, float s,
                  void* stream) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n4 = n / 4;
    const int64_t want = (n4 + (int64_t)kBlock * kUnroll - 1) / ((int64_t)kBlock * kUnroll);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * kBlocksPerCu));
    hipStream_t st = (hipStream_t)stream;
    if (n4 > 0) {
        if (kind == 1)
            hipLaunchKernelGGL(k_stream<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                               reinterpret_cast<const f4*>(a), reinterpret_cast<const f4*>(b),
                               reinterpret_cast<f4*>(c), n4, s);
        else
            hipLaunchKernelGGL(k_stream<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                               reinterpret_cast<const f4*>(a), reinterpret_cast<const f4*>(a),
                               reinterpret_cast<f4*>(c), n4, s);
    }
    if (n4 * 4 < n)
        hipLaunchKernelGGL(k_stream_tail, dim3(1), dim3(64), 0, st, a, kind == 1 ? b : a, c, n4 * 4,
                           n, s, kind == 1 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "stream launch failed: %s", hipGetErrorString(e));
    return FIPT_OK;
}

}  // namespace fipt
