// C ABI of libfipt (declared in include/fipt.h): argument validation,
// object lifetimes and kernel launches.  Every argument is checked before
// anything is enqueued; errors are reported through return codes and the
// calling thread's last-error text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "fipt_internal.hpp"

namespace fipt {

namespace {
thread_local char g_err[1024] = {0};
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

}  // namespace fipt

using namespace fipt;

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                              \
    } while (0)

namespace {

struct DeviceGuard {
    int prev = -1;
    int rc = FIPT_OK;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) {
            hipError_t e = hipSetDevice(dev);
            if (e != hipSuccess) rc = fail(FIPT_EHIP, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
        }
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename T>
int dev_alloc(T** p, size_t count, int64_t* bytes) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "hipMalloc(%zu): %s",
                    sizeof(T) * count, hipGetErrorString(e));
    if (bytes) *bytes += (int64_t)(sizeof(T) * count);
    return FIPT_OK;
}

void scene_free(fipt_scene s) {
    if (!s) return;
    if (s->d_nodes) (void)hipFree(s->d_nodes);
    if (s->d_tris) (void)hipFree(s->d_tris);
    if (s->d_rad) (void)hipFree(s->d_rad);
    if (s->d_vox) (void)hipFree(s->d_vox);
    if (s->d_vox_words) (void)hipFree(s->d_vox_words);
    if (s->d_vox_total) (void)hipFree(s->d_vox_total);
    if (s->d_vox_tiles) (void)hipFree(s->d_vox_tiles);
    if (s->d_order) (void)hipFree(s->d_order);
    if (s->d_leaf_of) (void)hipFree(s->d_leaf_of);
    if (s->d_emit) (void)hipFree(s->d_emit);
    if (s->d_emit_blocks) (void)hipFree(s->d_emit_blocks);
    if (s->refine_done) (void)hipEventDestroy(s->refine_done);
    if (s->d_tri_idx) (void)hipFree(s->d_tri_idx);
    if (s->d_counters) (void)hipFree(s->d_counters);
    for (hipEvent_t& e : s->slot_done)
        if (e) (void)hipEventDestroy(e);
    delete s;
}

int check_points(const fipt_points* pts, const char* name) {
    if (!pts) return fail(FIPT_EINVAL, "%s is NULL", name);
    if (!pts->planes || !pts->tri) return fail(FIPT_EINVAL, "%s has a NULL plane pointer", name);
    if (pts->n < 1 || pts->n > INT32_MAX)
        return fail(FIPT_EINVAL, "%s->n must be in [1, 2^31), got %lld", name, (long long)pts->n);
    if (pts->stride < pts->n)
        return fail(FIPT_EINVAL, "%s->stride (%lld) < n (%lld)", name, (long long)pts->stride,
                    (long long)pts->n);
    return FIPT_OK;
}

}  // namespace

namespace fipt {

int check_bake_params(const fipt_bake_params* p) {
    if (!p) return fail(FIPT_EINVAL, "params is NULL");
    if (p->spp_d < 1 || p->spp_d > 65536)
        return fail(FIPT_EINVAL, "spp_d must be in [1, 65536], got %d", p->spp_d);
    if (p->spp_s < 1 || p->spp_s > 65536)
        return fail(FIPT_EINVAL, "spp_s must be in [1, 65536], got %d", p->spp_s);
    if (p->n_levels < 1 || p->n_levels > FIPT_MAX_LEVELS)
        return fail(FIPT_EINVAL, "n_levels must be in [1, %d], got %d", FIPT_MAX_LEVELS, p->n_levels);
    for (int k = 0; k < p->n_levels; ++k) {
        const float s = p->sigma[k];
        if (!(s > 0.0f && s <= 1.0f)) return fail(FIPT_EINVAL, "sigma[%d] = %g outside (0, 1]", k, s);
        if (k > 0 && !(s > p->sigma[k - 1]))
            return fail(FIPT_EINVAL, "sigma must be strictly increasing (sigma[%d] = %g)", k, s);
    }
    if (!(p->ray_eps > 0.0f) || !std::isfinite(p->ray_eps))
        return fail(FIPT_EINVAL, "ray_eps must be positive and finite, got %g", p->ray_eps);
    if (p->flags != 0) return fail(FIPT_EINVAL, "flags must be 0");
    return FIPT_OK;
}

BakeLaunch make_bake_launch(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                            const fipt_shading* out) {
    BakeLaunch b;
    std::memset(&b, 0, sizeof(b));
    b.sc = s->view();
    b.pts = pts->planes;
    b.ptri = pts->tri;
    b.pts_stride = pts->stride;
    b.n = pts->n;
    b.p_offset = 0;
    b.out = out->planes;
    b.out_stride = out->stride;
    b.spp_d = p->spp_d;
    b.spp_s = p->spp_s;
    b.w_d = stratum_width(p->spp_d);
    b.w_s = stratum_width(p->spp_s);
    b.K = p->n_levels;
    for (int k = 0; k < FIPT_MAX_LEVELS; ++k) b.sigma[k] = k < p->n_levels ? p->sigma[k] : 1.0f;
    b.seed = p->seed;
    b.eps = p->ray_eps;
    return b;
}

}  // namespace fipt

extern "C" {

const char* fipt_last_error(void) { return g_err; }

int32_t fipt_version(void) { return 10000; }

int fipt_scene_create(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                      int32_t device, void* stream, fipt_scene* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!verts || !tris) return fail(FIPT_EINVAL, "verts/tris is NULL");
    if (n_verts < 3) return fail(FIPT_EINVAL, "n_verts must be >= 3, got %lld", (long long)n_verts);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(FIPT_EHIP, "no HIP device available");
    if (device < 0 || device >= ndev)
        return fail(FIPT_EINVAL, "device %d outside [0, %d)", device, ndev);
    HostBvh bvh;
    int rc = build_bvh(verts, n_verts, tris, n_tris, &bvh);
    if (rc) return rc;
    DeviceGuard g(device);
    if (g.rc) return g.rc;
    fipt_scene s = new fipt_scene_s();
    s->device = device;
    s->n_tris = n_tris;
    s->n_verts = n_verts;
    s->n_nodes = (int64_t)bvh.nodes4.size();
    s->max_depth = bvh.max_depth;
    s->box_scale = std::ldexp(1.0f, bvh.box_exp);
    for (int k = 0; k < 3; ++k) {
        s->bmin[k] = bvh.bmin[k];
        s->bmax[k] = bvh.bmax[k];
    }
    hipStream_t st = (hipStream_t)stream;
    if ((rc = dev_alloc(&s->d_nodes, bvh.nodes4.size(), &s->bytes)) ||
        (rc = dev_alloc(&s->d_tris, bvh.tris.size(), &s->bytes)) ||
        (rc = dev_alloc(&s->d_rad, bvh.tris.size(), &s->bytes)) ||
        (rc = dev_alloc(&s->d_order, bvh.order.size(), &s->bytes)) ||
        (rc = dev_alloc(&s->d_tri_idx, (size_t)(3 * n_tris), &s->bytes)) ||
        (rc = dev_alloc(&s->d_counters, (size_t)kBakeSlots * kXcdCount, &s->bytes)) ||
        (rc = dev_alloc(&s->d_leaf_of, (size_t)n_tris, &s->bytes)) ||
        (rc = dev_alloc(&s->d_emit, (size_t)n_tris + 1, &s->bytes)) ||
        (rc = dev_alloc(&s->d_emit_blocks, (size_t)((n_tris + 255) / 256), &s->bytes))) {
        scene_free(s);
        return rc;
    }
    {
        hipError_t e = hipEventCreateWithFlags(&s->refine_done, hipEventDisableTiming);
        if (e != hipSuccess) {
            scene_free(s);
            return fail(FIPT_EHIP, "scene events: %s", hipGetErrorString(e));
        }
    }
    std::vector<int32_t> leaf_of(bvh.order.size());
    for (size_t i = 0; i < bvh.order.size(); ++i) leaf_of[bvh.order[i]] = (int32_t)i;
    for (hipEvent_t& ev : s->slot_done) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            scene_free(s);
            return fail(FIPT_EHIP, "scene events: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = hipMemcpyAsync(s->d_nodes, bvh.nodes4.data(),
                                  sizeof(Bvh4Node) * bvh.nodes4.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_tris, bvh.tris.data(), sizeof(TriGeom) * bvh.tris.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_order, bvh.order.data(), sizeof(int32_t) * bvh.order.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_tri_idx, tris, sizeof(int32_t) * 3 * n_tris, hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_leaf_of, leaf_of.data(), sizeof(int32_t) * leaf_of.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host vectors go out of scope
    if (e != hipSuccess) {
        scene_free(s);
        return fail(FIPT_EHIP, "scene upload: %s", hipGetErrorString(e));
    }
    rc = launch_set_radiance(s->d_rad, s->d_order, s->d_tri_idx, n_tris, FIPT_CACHE_TRIANGLE,
                             nullptr, n_tris, nullptr, stream);
    if (rc) {
        scene_free(s);
        return rc;
    }
    *out = s;
    return FIPT_OK;
}

int fipt_scene_set_radiance(fipt_scene s, int32_t cache_kind, const float* cache, int64_t n_cache,
                            const float* emission, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    if (cache_kind != FIPT_CACHE_TRIANGLE && cache_kind != FIPT_CACHE_VERTEX)
        return fail(FIPT_EINVAL, "unknown cache kind %d", cache_kind);
    if (!cache) return fail(FIPT_EINVAL, "cache is NULL");
    const int64_t want = cache_kind == FIPT_CACHE_VERTEX ? s->n_verts : s->n_tris;
    if (n_cache != want)
        return fail(FIPT_EINVAL, "cache has %lld entries, scene needs %lld", (long long)n_cache,
                    (long long)want);
    if (s->refs.load() > 0)
        return fail(FIPT_EBUSY, "scene referenced by %d serving requests", s->refs.load());
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    int rc = launch_set_radiance(s->d_rad, s->d_order, s->d_tri_idx, s->n_tris, cache_kind, cache,
                                 n_cache, emission, stream);
    if (rc == FIPT_OK) s->cache_kind = cache_kind;
    return rc;
}

int fipt_scene_set_voxel_radiance(fipt_scene s, const float* cache, int64_t cache_stride,
                                  int32_t res, const float* bmin_host, const float* bmax_host,
                                  const float* emission, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    if (!cache || !bmin_host || !bmax_host) return fail(FIPT_EINVAL, "cache/bmin/bmax is NULL");
    if (res < 1 || res > kMaxVoxelRes)
        return fail(FIPT_EINVAL, "res must be in [1, %d], got %d", kMaxVoxelRes, res);
    const int64_t n_vox = (int64_t)res * res * res;
    if (cache_stride < n_vox) return fail(FIPT_EINVAL, "cache_stride < res^3");
    float scale[3];
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(bmin_host[a]) || !std::isfinite(bmax_host[a]) ||
            !(bmax_host[a] > bmin_host[a]))
            return fail(FIPT_EINVAL, "the box must be finite with bmin < bmax on every axis");
        scale[a] = (float)((double)res / ((double)bmax_host[a] - (double)bmin_host[a]));
        if (!std::isfinite(scale[a]) || !(scale[a] > 0.0f))
            return fail(FIPT_EINVAL, "the box is too thin for single precision");
    }
    // serving launches read the scene's radiance records, which this call
    // rewrites
    if (s->refs.load() > 0)
        return fail(FIPT_EBUSY, "scene referenced by %d serving requests", s->refs.load());
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n_bricks_axis = (res + 3) / 4;
    const int64_t n_words = n_bricks_axis * n_bricks_axis * n_bricks_axis;
    // the bake may still be reading the old grid: wait before replacing it;
    // until the new grid is complete the scene reads no voxel cache
    HIP_TRY(hipDeviceSynchronize());
    s->cache_kind = -1;
    if (!s->d_vox_total) {
        int rc = dev_alloc(&s->d_vox_total, 1, &s->bytes);
        if (rc) return rc;
    }
    if (s->vox_word_capacity < n_words) {
        const int64_t old_tiles = (s->vox_word_capacity + kVoxelScanTile - 1) / kVoxelScanTile;
        if (s->d_vox_words) {
            (void)hipFree(s->d_vox_words);
            (void)hipFree(s->d_vox_tiles);
            s->bytes -= 16 * s->vox_word_capacity + 4 * old_tiles;
            s->d_vox_words = nullptr;
            s->d_vox_tiles = nullptr;
            s->vox_word_capacity = 0;
        }
        int rc = dev_alloc(&s->d_vox_words, (size_t)n_words, &s->bytes);
        if (rc) return rc;
        rc = dev_alloc(&s->d_vox_tiles, (size_t)((n_words + kVoxelScanTile - 1) / kVoxelScanTile),
                       &s->bytes);
        if (rc) {
            (void)hipFree(s->d_vox_words);
            s->bytes -= 16 * n_words;
            s->d_vox_words = nullptr;
            return rc;
        }
        s->vox_word_capacity = n_words;
    }
    int rc = launch_voxel_words(s->d_vox_words, cache, cache_stride, res, s->d_vox_tiles,
                                s->d_vox_total, stream);
    if (rc) return rc;
    int64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, s->d_vox_total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (s->vox_capacity < std::max<int64_t>(total, 1)) {
        if (s->d_vox) {
            (void)hipFree(s->d_vox);
            s->bytes -= 16 * s->vox_capacity;
            s->d_vox = nullptr;
            s->vox_capacity = 0;
        }
        const int64_t cap = std::max<int64_t>(total, 1);
        rc = dev_alloc(&s->d_vox, (size_t)cap, &s->bytes);
        if (rc) return rc;
        s->vox_capacity = cap;
    }
    rc = launch_voxel_compact(s->d_vox, s->d_vox_words, cache, cache_stride, res, stream);
    if (rc) return rc;
    // corner values zero, emission as given
    rc = launch_set_radiance(s->d_rad, s->d_order, s->d_tri_idx, s->n_tris, FIPT_CACHE_TRIANGLE,
                             nullptr, s->n_tris, emission, stream);
    if (rc) return rc;
    s->vox_res = res;
    for (int a = 0; a < 3; ++a) {
        s->vox_lo[a] = bmin_host[a];
        s->vox_scale[a] = scale[a];
    }
    s->cache_kind = FIPT_CACHE_VOXEL;
    return FIPT_OK;
}

int fipt_scene_set_emission(fipt_scene s, const float* emission, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    if (!emission) return fail(FIPT_EINVAL, "emission is NULL");
    if (s->refs.load() > 0)
        return fail(FIPT_EBUSY, "scene referenced by %d serving requests", s->refs.load());
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    return launch_set_emission(s->d_rad, s->d_order, s->n_tris, emission, stream);
}

int fipt_scene_info_get(fipt_scene s, fipt_scene_info* out) {
    clear_error();
    if (!s || !out) return fail(FIPT_EINVAL, "scene/out is NULL");
    out->n_tris = s->n_tris;
    out->n_verts = s->n_verts;
    out->n_nodes = s->n_nodes;
    out->device_bytes = s->bytes;
    out->max_depth = s->max_depth;
    out->cache_kind = s->cache_kind;
    for (int k = 0; k < 3; ++k) {
        out->bmin[k] = s->bmin[k];
        out->bmax[k] = s->bmax[k];
    }
    return FIPT_OK;
}

int fipt_scene_destroy(fipt_scene s) {
    clear_error();
    if (!s) return FIPT_OK;
    if (s->refs.load() > 0) return fail(FIPT_EBUSY, "scene referenced by %d serving requests", s->refs.load());
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    (void)hipDeviceSynchronize();
    scene_free(s);
    return FIPT_OK;
}

int fipt_gen_points(fipt_scene s, const fipt_camera* cams, int32_t n_cams, const fipt_points* out,
                    void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    if (!cams || n_cams < 1 || n_cams > kMaxCameras)
        return fail(FIPT_EINVAL, "n_cams must be in [1, %d], got %d", kMaxCameras, n_cams);
    int rc = check_points(out, "out");
    if (rc) return rc;
    std::vector<int64_t> offs(n_cams + 1, 0);
    for (int c = 0; c < n_cams; ++c) {
        const fipt_camera& k = cams[c];
        if (k.width < 1 || k.height < 1)
            return fail(FIPT_EINVAL, "camera %d has size %dx%d", c, k.width, k.height);
        if (!(k.vfov_deg > 0.0f && k.vfov_deg < 180.0f))
            return fail(FIPT_EINVAL, "camera %d vfov %g outside (0, 180)", c, k.vfov_deg);
        const float f2 = k.fwd[0] * k.fwd[0] + k.fwd[1] * k.fwd[1] + k.fwd[2] * k.fwd[2];
        const float cx = k.fwd[1] * k.up[2] - k.fwd[2] * k.up[1];
        const float cy = k.fwd[2] * k.up[0] - k.fwd[0] * k.up[2];
        const float cz = k.fwd[0] * k.up[1] - k.fwd[1] * k.up[0];
        if (!(f2 > 0.0f) || !(cx * cx + cy * cy + cz * cz > 0.0f))
            return fail(FIPT_EINVAL, "camera %d: fwd is zero or parallel to up", c);
        offs[c + 1] = offs[c] + (int64_t)k.width * k.height;
    }
    if (offs[n_cams] != out->n)
        return fail(FIPT_EINVAL, "cameras have %lld pixels, out->n is %lld", (long long)offs[n_cams],
                    (long long)out->n);
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    CameraTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.n = n_cams;
    for (int c = 0; c < n_cams; ++c) tab.cam[c] = cams[c];
    for (int c = 0; c <= n_cams; ++c) tab.offset[c] = offs[c];
    return launch_gen_points(s->view(), tab, *out, stream);
}

int fipt_cast_rays(fipt_scene s, const float* rays, int64_t n, int64_t stride, int32_t* hit_tri,
                   float* hit_tuv, int64_t hit_stride, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    if (!rays || !hit_tri) return fail(FIPT_EINVAL, "rays/hit_tri is NULL");
    if (n < 1 || n > INT32_MAX) return fail(FIPT_EINVAL, "n must be in [1, 2^31), got %lld", (long long)n);
    if (stride < n) return fail(FIPT_EINVAL, "stride (%lld) < n (%lld)", (long long)stride, (long long)n);
    if (hit_tuv && hit_stride < n)
        return fail(FIPT_EINVAL, "hit_stride (%lld) < n (%lld)", (long long)hit_stride, (long long)n);
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    return launch_cast_rays(s->view(), rays, n, stride, hit_tri, hit_tuv, hit_stride, stream);
}

int fipt_lobe_uniforms(uint64_t seed, int64_t p0, int64_t n_points, int32_t lobe,
                       int32_t n_samples, float* out, void* stream) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    if (n_points < 1 || n_samples < 1 || n_points * (int64_t)n_samples > INT32_MAX)
        return fail(FIPT_EINVAL, "n_points x n_samples must be in [1, 2^31)");
    if (p0 < 0) return fail(FIPT_EINVAL, "p0 must be >= 0");
    if (lobe < 0 || lobe > FIPT_MAX_LEVELS) return fail(FIPT_EINVAL, "lobe must be in [0, %d]", FIPT_MAX_LEVELS);
    return launch_lobe_uniforms(seed, p0, n_points, lobe, n_samples, out, stream);
}

static int bake_common(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                       const fipt_shading* out, uint64_t* stats, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    int rc = check_points(pts, "pts");
    if (rc) return rc;
    if ((rc = check_bake_params(p))) return rc;
    if (!out || !out->planes) return fail(FIPT_EINVAL, "out is NULL");
    if (out->stride < pts->n)
        return fail(FIPT_EINVAL, "out->stride (%lld) < n (%lld)", (long long)out->stride,
                    (long long)pts->n);
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    BakeLaunch b = make_bake_launch(s, pts, p, out);
    // take the next counter slot; wait (on the stream) for its last user
    std::lock_guard<std::mutex> lk(s->slot_mu);
    const int k = s->next_slot;
    s->next_slot = (k + 1) % kBakeSlots;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamWaitEvent(st, s->slot_done[k], 0);
    if (e != hipSuccess) return fail(FIPT_EHIP, "bake slot wait: %s", hipGetErrorString(e));
    rc = launch_bake(b, s->d_counters + (size_t)k * kXcdCount, stats, stream);
    if (rc) return rc;
    e = hipEventRecord(s->slot_done[k], st);
    if (e != hipSuccess) return fail(FIPT_EHIP, "bake slot event: %s", hipGetErrorString(e));
    return FIPT_OK;
}

int fipt_bake(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
              const fipt_shading* out, void* stream) {
    return bake_common(s, pts, p, out, nullptr, stream);
}

int fipt_bake_traversal_stats(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                              const fipt_shading* out, uint64_t* stats_dev, void* stream) {
    if (!stats_dev) {
        clear_error();
        return fail(FIPT_EINVAL, "stats_dev is NULL");
    }
    return bake_common(s, pts, p, out, stats_dev, stream);
}

int fipt_refine(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                const fipt_refine_params* r, const fipt_shading* out, void* stream) {
    clear_error();
    if (!s) return fail(FIPT_EINVAL, "scene is NULL");
    int rc = check_points(pts, "pts");
    if (rc) return rc;
    if ((rc = check_bake_params(p))) return rc;
    if (!out || !out->planes) return fail(FIPT_EINVAL, "out is NULL");
    if (out->stride < pts->n)
        return fail(FIPT_EINVAL, "out->stride (%lld) < n (%lld)", (long long)out->stride,
                    (long long)pts->n);
    if (!r || !r->material) return fail(FIPT_EINVAL, "refine params or material grid is NULL");
    if (r->res < 2 || r->res > 1024) return fail(FIPT_EINVAL, "res must be in [2, 1024]");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(r->bmin[k]) || !std::isfinite(r->bmax[k]) || !(r->bmax[k] > r->bmin[k]))
            return fail(FIPT_EINVAL, "the material box must be finite with bmin < bmax");
    if (!std::isfinite(r->sigma_diffuse)) return fail(FIPT_EINVAL, "sigma_diffuse is not finite");
    if (r->max_vertices < 1 || r->max_vertices > 16)
        return fail(FIPT_EINVAL, "max_vertices must be in [1, 16], got %d", r->max_vertices);
    if (r->flags & ~FIPT_REFINE_BSDF_ONLY) return fail(FIPT_EINVAL, "unknown flags %d", r->flags);
    if (s->cache_kind == FIPT_CACHE_VOXEL)
        return fail(FIPT_EINVAL, "the refinement takes a per-triangle or per-vertex cache, not a voxel cache");
    DeviceGuard g(s->device);
    if (g.rc) return g.rc;
    BakeLaunch b = make_bake_launch(s, pts, p, out);
    hipStream_t st = (hipStream_t)stream;
    // refinements of one scene run in call order (they rewrite its emitter
    // list); the work counters come from the bake's slot ring
    std::lock_guard<std::mutex> rk(s->refine_mu);
    hipError_t e = hipStreamWaitEvent(st, s->refine_done, 0);
    if (e != hipSuccess) return fail(FIPT_EHIP, "refine wait: %s", hipGetErrorString(e));
    rc = launch_emitter_list(s->d_rad, s->d_leaf_of, s->n_tris, s->d_emit_blocks, s->d_emit,
                             s->d_emit + s->n_tris, stream);
    if (rc) return rc;
    RefineLaunch rl;
    rl.grid = r->material;
    rl.res = r->res;
    for (int k = 0; k < 3; ++k) {
        rl.bmin[k] = r->bmin[k];
        rl.bmax[k] = r->bmax[k];
    }
    rl.sigma_diffuse = r->sigma_diffuse;
    rl.max_vertices = r->max_vertices;
    rl.flags = r->flags;
    rl.emit = s->d_emit;
    rl.n_emit = s->d_emit + s->n_tris;
    {
        std::lock_guard<std::mutex> lk(s->slot_mu);
        const int k = s->next_slot;
        s->next_slot = (k + 1) % kBakeSlots;
        e = hipStreamWaitEvent(st, s->slot_done[k], 0);
        if (e != hipSuccess) return fail(FIPT_EHIP, "refine slot wait: %s", hipGetErrorString(e));
        rc = launch_refine(b, rl, s->d_counters + (size_t)k * kXcdCount, stream);
        if (rc) return rc;
        e = hipEventRecord(s->slot_done[k], st);
        if (e != hipSuccess) return fail(FIPT_EHIP, "refine slot event: %s", hipGetErrorString(e));
    }
    e = hipEventRecord(s->refine_done, st);
    if (e != hipSuccess) return fail(FIPT_EHIP, "refine event: %s", hipGetErrorString(e));
    return FIPT_OK;
}

namespace {
int check_render_loss(const fipt_shading* sh, int64_t n, int32_t n_levels, const float* sigma_host,
                      const float* material, int64_t mat_stride, const float* observed,
                      int64_t obs_stride, int32_t tonemap, const double* loss_dev,
                      const float* grad_dev, int64_t grad_stride, const float* Lr_dev,
                      int64_t lr_stride) {
    if (!sh || !sh->planes) return fail(FIPT_EINVAL, "shading is NULL");
    if (n < 1) return fail(FIPT_EINVAL, "n must be >= 1, got %lld", (long long)n);
    if (n_levels < 2 || n_levels > FIPT_MAX_LEVELS)
        return fail(FIPT_EINVAL, "n_levels must be in [2, %d], got %d", FIPT_MAX_LEVELS, n_levels);
    if (!sigma_host) return fail(FIPT_EINVAL, "sigma is NULL");
    for (int k = 0; k < n_levels; ++k) {
        if (!std::isfinite(sigma_host[k])) return fail(FIPT_EINVAL, "sigma[%d] is not finite", k);
        if (k > 0 && !(sigma_host[k] > sigma_host[k - 1]))
            return fail(FIPT_EINVAL, "sigma must be strictly increasing");
    }
    if (!material || !observed || !loss_dev)
        return fail(FIPT_EINVAL, "material/observed/loss is NULL");
    if (sh->stride < n || mat_stride < n || obs_stride < n)
        return fail(FIPT_EINVAL, "a stride is smaller than n");
    if (grad_dev && grad_stride < n) return fail(FIPT_EINVAL, "grad_stride < n");
    if (Lr_dev && lr_stride < n) return fail(FIPT_EINVAL, "lr_stride < n");
    if (tonemap != FIPT_TONEMAP_NONE && tonemap != FIPT_TONEMAP_LOG_SRGB)
        return fail(FIPT_EINVAL, "unknown tonemap %d", tonemap);
    return FIPT_OK;
}
}  // namespace

int fipt_render_loss(const fipt_shading* sh, int64_t n, int32_t n_levels, const float* sigma_host,
                     const float* material, int64_t mat_stride, const float* observed,
                     int64_t obs_stride, int32_t tonemap, double* loss_dev, float* grad_dev,
                     int64_t grad_stride, float* Lr_dev, int64_t lr_stride, void* stream) {
    clear_error();
    int rc = check_render_loss(sh, n, n_levels, sigma_host, material, mat_stride, observed,
                               obs_stride, tonemap, loss_dev, grad_dev, grad_stride, Lr_dev,
                               lr_stride);
    if (rc) return rc;
    return launch_render_loss(sh->planes, sh->stride, n, n_levels, sigma_host, material, mat_stride,
                              observed, obs_stride, tonemap, loss_dev, loss_dev + 1, grad_dev,
                              grad_stride, Lr_dev, lr_stride, nullptr, stream);
}

int fipt_render_loss_noalloc(const fipt_shading* sh, int64_t n, int32_t n_levels,
                             const float* sigma_host, const float* material, int64_t mat_stride,
                             const float* observed, int64_t obs_stride, int32_t tonemap,
                             double* loss_dev, float* grad_dev, int64_t grad_stride,
                             float* Lr_dev, int64_t lr_stride, void* stream) {
    clear_error();
    int rc = check_render_loss(sh, n, n_levels, sigma_host, material, mat_stride, observed,
                               obs_stride, tonemap, loss_dev, grad_dev, grad_stride, Lr_dev,
                               lr_stride);
    if (rc) return rc;
    double* partials = nullptr;
    int64_t capacity = 0;
    if ((rc = render_loss_scratch(&partials, &capacity))) return rc;
    const int64_t need = render_loss_partials(n);
    if (need > capacity)
        return fail(FIPT_EINVAL, "render loss needs %lld partial sums, the static array holds %lld",
                    (long long)need, (long long)capacity);
    return launch_render_loss(sh->planes, sh->stride, n, n_levels, sigma_host, material, mat_stride,
                              observed, obs_stride, tonemap, loss_dev, partials, grad_dev,
                              grad_stride, Lr_dev, lr_stride, nullptr, stream);
}

int fipt_render_loss_masked(const fipt_shading* sh, int64_t n, int32_t n_levels,
                            const float* sigma_host, const float* material, int64_t mat_stride,
                            const float* observed, int64_t obs_stride, const float* alpha,
                            int32_t tonemap, double lambda_d, double* loss_dev, float* grad_dev,
                            int64_t grad_stride, float* grad_alpha_dev, float* Lr_dev,
                            int64_t lr_stride, void* stream) {
    clear_error();
    int rc = check_render_loss(sh, n, n_levels, sigma_host, material, mat_stride, observed,
                               obs_stride, tonemap, loss_dev, grad_dev, grad_stride, Lr_dev,
                               lr_stride);
    if (rc) return rc;
    if (!std::isfinite(lambda_d) || lambda_d < 0.0)
        return fail(FIPT_EINVAL, "lambda_d must be finite and >= 0");
    const RenderLossMask mask{alpha, grad_alpha_dev, lambda_d};
    return launch_render_loss(sh->planes, sh->stride, n, n_levels, sigma_host, material, mat_stride,
                              observed, obs_stride, tonemap, loss_dev, loss_dev + 1, grad_dev,
                              grad_stride, Lr_dev, lr_stride, &mask, stream);
}

int fipt_scale_by(const float* x, int64_t n, const double* factor_dev, float* out, void* stream) {
    clear_error();
    if (!x || !factor_dev || !out) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 0) return fail(FIPT_EINVAL, "n must be >= 0");
    if (n == 0) return FIPT_OK;
    return launch_scale_by(x, n, factor_dev, out, stream);
}

int fipt_hbm_stream(int32_t kind, const float* a, const float* b, float* c, int64_t n, float s,
                    void* stream) {
    clear_error();
    if (kind != 0 && kind != 1) return fail(FIPT_EINVAL, "kind must be 0 (copy) or 1 (triad)");
    if (!a || !c || (kind == 1 && !b)) return fail(FIPT_EINVAL, "NULL argument");
    if (n < 1) return fail(FIPT_EINVAL, "n must be >= 1");
    const uintptr_t mis = (reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(c) |
                           (kind == 1 ? reinterpret_cast<uintptr_t>(b) : 0)) & 15u;
    if (mis) return fail(FIPT_EINVAL, "arrays must be 16-byte aligned");
    return launch_stream(kind, a, b, c, n, s, stream);
}

int fipt_grid_gather(const float* grid, int32_t channels, int32_t res, const float* bmin_host,
                     const float* bmax_host, const float* pos, int64_t pos_stride, int64_t n,
                     float* out, int64_t out_stride, void* stream) {
    clear_error();
    if (!grid || !pos || !out || !bmin_host || !bmax_host) return fail(FIPT_EINVAL, "NULL argument");
    if (channels < 1 || channels > 8) return fail(FIPT_EINVAL, "channels must be in [1, 8]");
    if (res < 2 || res > 1024) return fail(FIPT_EINVAL, "res must be in [2, 1024]");
    if (n < 1) return fail(FIPT_EINVAL, "n must be >= 1");
    if (pos_stride < n || out_stride < n) return fail(FIPT_EINVAL, "a stride is smaller than n");
    for (int k = 0; k < 3; ++k)
        if (!(bmax_host[k] > bmin_host[k])) return fail(FIPT_EINVAL, "empty grid box on axis %d", k);
    return launch_grid_gather(grid, channels, res, bmin_host, bmax_host, pos, pos_stride, n, out,
                              out_stride, stream);
}

}  // extern "C"
