"""Python binding of libfipt (include/fipt.h).

Argument marshalling only: every function here checks tensor shapes, dtypes
and devices, then calls the C entry point of the same name (``fipt_*``) on
torch's current HIP stream.  All computation happens in the library's HIP
kernels; nothing falls back to the CPU.  If libfipt.so has not been built,
loading fails with an error naming the build step.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# FIPT_LIBRARY may point at another build of the same library
LIB_PATH = os.environ.get("FIPT_LIBRARY", os.path.join(HERE, "libfipt.so"))

OK, EINVAL, ENOMEM, EHIP, EBUSY, EAGAIN, ECANCELED = 0, -1, -2, -3, -4, -5, -6
MAX_LEVELS = 16
LOSS_SLOTS = 2049
CACHE_TRIANGLE, CACHE_VERTEX, CACHE_VOXEL = 0, 1, 2
TONEMAP_NONE, TONEMAP_LOG_SRGB = 0, 1

# every entry point declared in include/fipt.h
EXPORTS = (
    "fipt_last_error", "fipt_version", "fipt_scene_create", "fipt_scene_set_radiance",
    "fipt_scene_set_emission", "fipt_scene_info_get", "fipt_bvh_validate", "fipt_scene_destroy",
    "fipt_cast_rays", "fipt_gen_points",
    "fipt_bake", "fipt_lobe_uniforms", "fipt_bake_traversal_stats", "fipt_refine", "fipt_render_loss",
    "fipt_render_loss_noalloc", "fipt_render_loss_masked", "fipt_scale_by", "fipt_hbm_stream",
    "fipt_grid_gather", "fipt_grid_plan_create", "fipt_grid_plan_destroy", "fipt_grid_scatter",
    "fipt_grid_plan_order", "fipt_grid_plan_permute", "fipt_grid_render_loss",
    "fipt_emission_plan_create", "fipt_emission_plan_destroy", "fipt_emission_median",
    "fipt_scene_set_voxel_radiance", "fipt_voxel_plan_create", "fipt_voxel_plan_destroy",
    "fipt_voxel_pool", "fipt_hashgrid_forward", "fipt_hashgrid_workspace_floats",
    "fipt_hashgrid_plan_create", "fipt_hashgrid_plan_destroy", "fipt_hashgrid_backward",
    "fipt_hashgrid_forward_save", "fipt_hashgrid_backward_saved",
    "fipt_server_create", "fipt_server_submit", "fipt_server_poll", "fipt_server_wait",
    "fipt_server_result", "fipt_server_release", "fipt_server_cancel", "fipt_server_stats_get",
    "fipt_server_destroy",
)


class FiptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fipt error {code}: {msg}")
        self.code = code


class Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("fwd", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class Points(C.Structure):
    _fields_ = [("planes", C.c_void_p), ("tri", C.c_void_p), ("n", C.c_int64),
                ("stride", C.c_int64)]


class Shading(C.Structure):
    _fields_ = [("planes", C.c_void_p), ("stride", C.c_int64)]


class BakeParams(C.Structure):
    _fields_ = [("spp_d", C.c_int32), ("spp_s", C.c_int32), ("n_levels", C.c_int32),
                ("sigma", C.c_float * MAX_LEVELS), ("seed", C.c_uint64), ("ray_eps", C.c_float),
                ("flags", C.c_int32)]


class RefineParams(C.Structure):
    _fields_ = [("material", C.c_void_p), ("res", C.c_int32), ("bmin", C.c_float * 3),
                ("bmax", C.c_float * 3), ("sigma_diffuse", C.c_float), ("max_vertices", C.c_int32),
                ("flags", C.c_int32)]


REFINE_BSDF_ONLY = 1


class SceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_verts", C.c_int64), ("n_nodes", C.c_int64),
                ("device_bytes", C.c_int64), ("max_depth", C.c_int32), ("cache_kind", C.c_int32),
                ("bmin", C.c_float * 3), ("bmax", C.c_float * 3)]


class ServerStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("tiles", C.c_int64), ("samples", C.c_int64),
                ("completed", C.c_int64), ("pool_in_use", C.c_int64), ("queued", C.c_int64),
                ("inflight", C.c_int64)]


_lib = None
_vp, _i32, _i64, _u64, _f32p = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.POINTER(C.c_float)


def lib():
    """Load libfipt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "fipt_last_error": (C.c_char_p, []),
        "fipt_version": (_i32, []),
        "fipt_scene_create": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _vp, C.POINTER(_vp)]),
        "fipt_scene_set_radiance": (C.c_int, [_vp, _i32, _vp, _i64, _vp, _vp]),
        "fipt_scene_set_voxel_radiance": (C.c_int, [_vp, _vp, _i64, _i32, _f32p, _f32p, _vp, _vp]),
        "fipt_voxel_plan_create": (C.c_int, [_vp, _i64, _i32, _f32p, _f32p, _i32, C.POINTER(_vp)]),
        "fipt_voxel_plan_destroy": (C.c_int, [_vp]),
        "fipt_voxel_pool": (C.c_int, [_vp, _vp, _i64, _vp, _i64, _vp]),
        "fipt_hashgrid_forward": (C.c_int, [_vp, _vp, _i64, _i64, _f32p, _f32p, _vp, _i64, _vp]),
        "fipt_hashgrid_workspace_floats": (_i64, [_i64]),
        "fipt_hashgrid_plan_create": (C.c_int, [_vp, _i64, _i64, _f32p, _f32p, _vp, C.POINTER(_vp)]),
        "fipt_hashgrid_plan_destroy": (C.c_int, [_vp]),
        "fipt_hashgrid_backward": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp]),
        "fipt_hashgrid_forward_save": (C.c_int, [_vp, _vp, _i64, _i64, _f32p, _f32p, _vp, _i64, _vp,
                                                 _i64, _vp]),
        "fipt_hashgrid_backward_saved": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp]),
        "fipt_scene_set_emission": (C.c_int, [_vp, _vp, _vp]),
        "fipt_scene_info_get": (C.c_int, [_vp, C.POINTER(SceneInfo)]),
        "fipt_scene_destroy": (C.c_int, [_vp]),
        "fipt_bvh_validate": (C.c_int, [_vp, _i64, _vp, _i64, C.POINTER(_i64), C.POINTER(_i32)]),
        "fipt_cast_rays": (C.c_int, [_vp, _vp, _i64, _i64, _vp, _vp, _i64, _vp]),
        "fipt_lobe_uniforms": (C.c_int, [_u64, _i64, _i64, _i32, _i32, _vp, _vp]),
        "fipt_gen_points": (C.c_int, [_vp, C.POINTER(Camera), _i32, C.POINTER(Points), _vp]),
        "fipt_bake": (C.c_int, [_vp, C.POINTER(Points), C.POINTER(BakeParams), C.POINTER(Shading), _vp]),
        "fipt_refine": (C.c_int, [_vp, C.POINTER(Points), C.POINTER(BakeParams), C.POINTER(RefineParams),
                                  C.POINTER(Shading), _vp]),
        "fipt_bake_traversal_stats": (C.c_int, [_vp, C.POINTER(Points), C.POINTER(BakeParams),
                                                C.POINTER(Shading), _vp, _vp]),
        "fipt_render_loss": (C.c_int, [C.POINTER(Shading), _i64, _i32, _f32p, _vp, _i64, _vp, _i64,
                                       _i32, _vp, _vp, _i64, _vp, _i64, _vp]),
        "fipt_render_loss_noalloc": (C.c_int, [C.POINTER(Shading), _i64, _i32, _f32p, _vp, _i64, _vp,
                                               _i64, _i32, _vp, _vp, _i64, _vp, _i64, _vp]),
        "fipt_render_loss_masked": (C.c_int, [C.POINTER(Shading), _i64, _i32, _f32p, _vp, _i64, _vp,
                                              _i64, _vp, _i32, C.c_double, _vp, _vp, _i64, _vp, _vp,
                                              _i64, _vp]),
        "fipt_scale_by": (C.c_int, [_vp, _i64, _vp, _vp, _vp]),
        "fipt_hbm_stream": (C.c_int, [_i32, _vp, _vp, _vp, _i64, C.c_float, _vp]),
        "fipt_grid_gather": (C.c_int, [_vp, _i32, _i32, _f32p, _f32p, _vp, _i64, _i64, _vp, _i64, _vp]),
        "fipt_grid_plan_create": (C.c_int, [_vp, _i64, _i32, _f32p, _f32p, _i32, C.POINTER(_vp)]),
        "fipt_grid_plan_destroy": (C.c_int, [_vp]),
        "fipt_grid_scatter": (C.c_int, [_vp, _vp, _i32, _i64, _vp, _vp]),
        "fipt_grid_plan_order": (C.c_int, [_vp, _vp]),
        "fipt_grid_plan_permute": (C.c_int, [_vp, _vp, _i32, _i64, _vp, _i64, _vp]),
        "fipt_grid_render_loss": (C.c_int, [_vp, _vp, C.POINTER(Shading), _i32, _f32p, _vp, _i64, _i32,
                                            _vp, _vp, _vp, _i64, _vp]),
        "fipt_emission_plan_create": (C.c_int, [_vp, _i64, _i64, _i32, C.POINTER(_vp)]),
        "fipt_emission_plan_destroy": (C.c_int, [_vp]),
        "fipt_emission_median": (C.c_int, [_vp, _vp, _i64, _vp, _vp, _i64, _vp]),
        "fipt_server_create": (C.c_int, [_i32, _i64, _i32, _i64, C.POINTER(_vp)]),
        "fipt_server_submit": (C.c_int, [_vp, _vp, C.POINTER(Points), C.POINTER(BakeParams),
                                         C.POINTER(_u64)]),
        "fipt_server_poll": (C.c_int, [_vp, _u64]),
        "fipt_server_wait": (C.c_int, [_vp, _u64, _i64]),
        "fipt_server_result": (C.c_int, [_vp, _u64, C.POINTER(Shading), C.POINTER(_i64),
                                         C.POINTER(_i64), C.POINTER(_i64)]),
        "fipt_server_release": (C.c_int, [_vp, _u64]),
        "fipt_server_cancel": (C.c_int, [_vp, _u64]),
        "fipt_server_stats_get": (C.c_int, [_vp, C.POINTER(ServerStats)]),
        "fipt_server_destroy": (C.c_int, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise FiptError(rc, lib().fipt_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _need(t: torch.Tensor, shape, name: str):
    """Reject a caller buffer whose shape differs from what the kernel writes
    or reads (the C entry points take bare pointers)."""
    if not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(shape):
        got = tuple(t.shape) if isinstance(t, torch.Tensor) else type(t).__name__
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {got}")


def _f32_array(v, n):
    a = (C.c_float * n)()
    for i, x in enumerate(v):
        a[i] = float(x)
    return a


def version() -> int:
    return int(lib().fipt_version())


# --------------------------------------------------------------------------
# scene
# --------------------------------------------------------------------------
class Scene:
    """Triangle mesh + BVH + radiance records resident on one GPU."""

    def __init__(self, verts, tris, device: int = 0):
        import numpy as np
        v = np.ascontiguousarray(verts, dtype=np.float32)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        h = C.c_void_p()
        with torch.cuda.device(device):
            _check(lib().fipt_scene_create(v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0],
                                           device, _stream(), C.byref(h)))
        self.handle = h
        self.device = device
        self.n_tris = int(t.shape[0])
        self.n_verts = int(v.shape[0])

    def set_radiance(self, cache: torch.Tensor, kind: int, emission: torch.Tensor = None):
        """cache: [3, n] float32 GPU (n = triangles or vertices by kind);
        emission: [3, n_tris] float32 GPU or None."""
        ep = _dev(emission, torch.float32, "emission") if emission is not None else None
        if emission is not None and tuple(emission.shape) != (3, self.n_tris):
            raise ValueError("emission must be [3, n_tris]")
        _check(lib().fipt_scene_set_radiance(self.handle, kind, _dev(cache, torch.float32, "cache"),
                                             cache.shape[1], ep, _stream()))

    def set_voxel_radiance(self, cache: torch.Tensor, res: int, bmin, bmax,
                           emission: torch.Tensor = None):
        """Voxel-grid radiance cache (Sec. 4.2): cache [3, res^3] float32 GPU
        (x fastest) over the box [bmin, bmax]; emission [3, n_tris] or None."""
        if cache.dim() != 2 or cache.shape[0] != 3 or cache.shape[1] != res ** 3:
            raise ValueError(f"cache must be [3, {res ** 3}], got {tuple(cache.shape)}")
        if emission is not None and tuple(emission.shape) != (3, self.n_tris):
            raise ValueError("emission must be [3, n_tris]")
        ep = _dev(emission, torch.float32, "emission") if emission is not None else None
        _check(lib().fipt_scene_set_voxel_radiance(
            self.handle, _dev(cache, torch.float32, "cache"), cache.shape[1], int(res),
            _f32_array(bmin, 3), _f32_array(bmax, 3), ep, _stream()))

    def set_emission(self, emission: torch.Tensor):
        if tuple(emission.shape) != (3, self.n_tris):
            raise ValueError("emission must be [3, n_tris]")
        _check(lib().fipt_scene_set_emission(self.handle, _dev(emission, torch.float32, "emission"),
                                             _stream()))

    def info(self) -> SceneInfo:
        out = SceneInfo()
        _check(lib().fipt_scene_info_get(self.handle, C.byref(out)))
        return out

    def destroy(self):
        if self.handle:
            _check(lib().fipt_scene_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_scene_destroy(self.handle)
        except Exception:
            pass


def fipt_bvh_validate(verts, tris):
    """Host-only: build and verify the BVH of a mesh; returns (nodes, depth)."""
    import numpy as np
    v = np.ascontiguousarray(verts, dtype=np.float32)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    nn, dd = C.c_int64(), C.c_int32()
    _check(lib().fipt_bvh_validate(v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0],
                                   C.byref(nn), C.byref(dd)))
    return nn.value, dd.value


def make_points(planes: torch.Tensor, tri: torch.Tensor) -> Points:
    if planes.dim() != 2 or planes.shape[0] != 9:
        raise ValueError("point planes must be [9, n]")
    if tri.shape != (planes.shape[1],):
        raise ValueError("tri must be [n]")
    return Points(_dev(planes, torch.float32, "planes"), _dev(tri, torch.int32, "tri"),
                  planes.shape[1], planes.shape[1])


def make_params(spp_d: int, spp_s: int, sigma, seed: int, ray_eps: float = 1e-4) -> BakeParams:
    p = BakeParams()
    p.spp_d = int(spp_d)
    p.spp_s = int(spp_s)
    # the C ABI validates n_levels (an over-long table is rejected there)
    p.n_levels = len(sigma)
    p.sigma = _f32_array(list(sigma)[:MAX_LEVELS], MAX_LEVELS)
    p.seed = int(seed)
    p.ray_eps = float(ray_eps)
    p.flags = 0
    return p


def fipt_cast_rays(scene: Scene, rays: torch.Tensor, want_tuv: bool = True):
    """rays: float32 GPU tensor [6, n] (origin xyz, direction xyz).  Returns
    (tri [n] int32: original triangle index or -1, tuv [3, n] float32 or
    None) of the closest hits."""
    if rays.dim() != 2 or rays.shape[0] != 6:
        raise ValueError("rays must be [6, n]")
    n = rays.shape[1]
    tri = torch.empty((n,), dtype=torch.int32, device=rays.device)
    tuv = torch.empty((3, n), dtype=torch.float32, device=rays.device) if want_tuv else None
    _check(lib().fipt_cast_rays(scene.handle, _dev(rays, torch.float32, "rays"), n, rays.stride(0),
                                _dev(tri, torch.int32, "tri"),
                                _dev(tuv, torch.float32, "tuv") if want_tuv else None, n,
                                _stream()))
    return tri, tuv


def fipt_lobe_uniforms(seed: int, p0: int, n_points: int, lobe: int, n_samples: int,
                       device: int = 0) -> torch.Tensor:
    """The bake's stratified uniforms for lobe ``lobe`` with n_samples
    samples, samples 0..n_samples-1 of the points p0..p0+n_points-1: float32
    GPU tensor [2, n_points, n_samples]."""
    out = torch.empty((2, n_points, n_samples), dtype=torch.float32, device=torch.device("cuda", device))
    _check(lib().fipt_lobe_uniforms(int(seed) & ((1 << 64) - 1), int(p0), int(n_points), int(lobe),
                                    int(n_samples), _dev(out, torch.float32, "out"), _stream()))
    return out


def fipt_gen_points(scene: Scene, cameras, planes: torch.Tensor = None, tri: torch.Tensor = None):
    """cameras: list of synth.Camera-like objects (pos, fwd, up, vfov_deg,
    width, height).  Returns (planes [9, n], tri [n]) GPU tensors."""
    n = sum(c.width * c.height for c in cameras)
    dev = torch.device("cuda", scene.device)
    if planes is None:
        planes = torch.empty((9, n), dtype=torch.float32, device=dev)
    if tri is None:
        tri = torch.empty((n,), dtype=torch.int32, device=dev)
    pts = make_points(planes, tri)
    # at most 48 cameras per call: offset the output pointers for more
    first = 0
    for c0 in range(0, len(cameras), 48):
        group = cameras[c0:c0 + 48]
        arr = (Camera * len(group))()
        cnt = 0
        for k, c in enumerate(group):
            arr[k].pos = _f32_array(c.pos, 3)
            arr[k].fwd = _f32_array(c.fwd, 3)
            arr[k].up = _f32_array(c.up, 3)
            arr[k].vfov_deg = float(c.vfov_deg)
            arr[k].width = int(c.width)
            arr[k].height = int(c.height)
            cnt += c.width * c.height
        sub = Points(pts.planes + 4 * first, pts.tri + 4 * first, cnt, n)
        _check(lib().fipt_gen_points(scene.handle, arr, len(group), C.byref(sub), _stream()))
        first += cnt
    return planes, tri


def fipt_bake(scene: Scene, planes: torch.Tensor, tri: torch.Tensor, spp_d: int, spp_s: int,
              sigma, seed: int, ray_eps: float = 1e-4, out: torch.Tensor = None,
              stats: torch.Tensor = None):
    """Bake Ld, Ls0[K], Ls1[K] for the points; returns [3 + 6K, n] float32.
    If ``stats`` (int64 GPU tensor of 7) is given, the instrumented kernel
    adds rays, nodes, triangles, hits, node-loop and triangle-loop
    wavefront steps to it."""
    if stats is not None and tuple(stats.shape) != (7,):
        raise ValueError("stats must be an int64 tensor of 7")
    K = len(sigma)
    n = planes.shape[1]
    if out is None:
        out = torch.empty((3 + 6 * K, n), dtype=torch.float32, device=planes.device)
    if out.shape[0] != 3 + 6 * K or out.shape[1] < n:
        raise ValueError("out must be [3 + 6K, >= n]")
    pts = make_points(planes, tri)
    par = make_params(spp_d, spp_s, sigma, seed, ray_eps)
    sh = Shading(_dev(out, torch.float32, "out"), out.shape[1])
    if stats is None:
        _check(lib().fipt_bake(scene.handle, C.byref(pts), C.byref(par), C.byref(sh), _stream()))
    else:
        _check(lib().fipt_bake_traversal_stats(scene.handle, C.byref(pts), C.byref(par), C.byref(sh),
                                               _dev(stats, torch.int64, "stats"), _stream()))
    return out


def fipt_refine(scene: Scene, planes: torch.Tensor, tri: torch.Tensor, spp_d: int, spp_s: int,
                sigma, seed: int, material: torch.Tensor, bmin, bmax, sigma_diffuse: float = 0.6,
                max_vertices: int = 8, flags: int = 0, ray_eps: float = 1e-4,
                out: torch.Tensor = None):
    """Refined shading terms (stage 3): the bake's samples, paths grown
    through glossy hits of the material grid [5, R, R, R] (a_r, a_g, a_b,
    sigma, m) over the box [bmin, bmax]; returns [3 + 6K, n] float32."""
    K = len(sigma)
    n = planes.shape[1]
    R = material.shape[-1]
    _need(material, (5, R, R, R), "material")
    if out is None:
        out = torch.empty((3 + 6 * K, n), dtype=torch.float32, device=planes.device)
    if out.shape[0] != 3 + 6 * K or out.shape[1] < n:
        raise ValueError("out must be [3 + 6K, >= n]")
    pts = make_points(planes, tri)
    par = make_params(spp_d, spp_s, sigma, seed, ray_eps)
    rp = RefineParams()
    rp.material = _dev(material, torch.float32, "material")
    rp.res = int(R)
    rp.bmin = (C.c_float * 3)(*[float(v) for v in bmin])
    rp.bmax = (C.c_float * 3)(*[float(v) for v in bmax])
    rp.sigma_diffuse = float(sigma_diffuse)
    rp.max_vertices = int(max_vertices)
    rp.flags = int(flags)
    sh = Shading(_dev(out, torch.float32, "out"), out.shape[1])
    _check(lib().fipt_refine(scene.handle, C.byref(pts), C.byref(par), C.byref(rp), C.byref(sh),
                             _stream()))
    return out


# --------------------------------------------------------------------------
# factored re-render + loss
# --------------------------------------------------------------------------
def fipt_render_loss(shading: torch.Tensor, material: torch.Tensor, observed: torch.Tensor, sigma,
                     tonemap: int = TONEMAP_NONE, want_grad: bool = True, want_lr: bool = False,
                     loss_buf: torch.Tensor = None, grad: torch.Tensor = None, lr: torch.Tensor = None):
    """Returns (loss_buf, grad, Lr): loss_buf[0] is the loss (float64 GPU);
    grad [5, n] and Lr [3, n] float32 GPU (or None)."""
    K = len(sigma)
    n = material.shape[1]
    if shading.shape[0] != 3 + 6 * K or shading.shape[1] != n:
        raise ValueError("shading must be [3 + 6K, n]")
    if material.shape[0] != 5 or observed.shape != (3, n):
        raise ValueError("material must be [5, n] and observed [3, n]")
    dev = material.device
    if loss_buf is None:
        loss_buf = torch.empty((LOSS_SLOTS,), dtype=torch.float64, device=dev)
    _need(loss_buf, (LOSS_SLOTS,), "loss_buf")
    if want_grad and grad is None:
        grad = torch.empty((5, n), dtype=torch.float32, device=dev)
    if want_grad:
        _need(grad, (5, n), "grad")
    if want_lr and lr is None:
        lr = torch.empty((3, n), dtype=torch.float32, device=dev)
    if want_lr:
        _need(lr, (3, n), "lr")
    sh = Shading(_dev(shading, torch.float32, "shading"), n)
    sig = _f32_array(sigma, K)
    _check(lib().fipt_render_loss(
        C.byref(sh), n, K, sig, _dev(material, torch.float32, "material"), n,
        _dev(observed, torch.float32, "observed"), n, int(tonemap),
        _dev(loss_buf, torch.float64, "loss_buf"),
        _dev(grad, torch.float32, "grad") if want_grad else None, n,
        _dev(lr, torch.float32, "lr") if want_lr else None, n, _stream()))
    return loss_buf, (grad if want_grad else None), (lr if want_lr else None)


def fipt_render_loss_noalloc(shading: torch.Tensor, material: torch.Tensor, observed: torch.Tensor,
                             sigma, loss: torch.Tensor, grad: torch.Tensor = None,
                             lr: torch.Tensor = None, tonemap: int = TONEMAP_NONE):
    """fipt_render_loss with every buffer supplied by the caller and nothing
    allocated, here or in the library: loss [1] float64 GPU receives the
    loss, grad [5, n] and Lr [3, n] float32 GPU (or None) as for
    fipt_render_loss.  Calls that overlap on one GPU race (see fipt.h)."""
    K = len(sigma)
    n = material.shape[1]
    if shading.shape[0] != 3 + 6 * K or shading.shape[1] != n:
        raise ValueError("shading must be [3 + 6K, n]")
    if material.shape[0] != 5 or observed.shape != (3, n):
        raise ValueError("material must be [5, n] and observed [3, n]")
    _need(loss, (1,), "loss")
    if grad is not None:
        _need(grad, (5, n), "grad")
    if lr is not None:
        _need(lr, (3, n), "lr")
    sh = Shading(_dev(shading, torch.float32, "shading"), n)
    sig = _f32_array(sigma, K)
    _check(lib().fipt_render_loss_noalloc(
        C.byref(sh), n, K, sig, _dev(material, torch.float32, "material"), n,
        _dev(observed, torch.float32, "observed"), n, int(tonemap),
        _dev(loss, torch.float64, "loss"),
        _dev(grad, torch.float32, "grad") if grad is not None else None, n,
        _dev(lr, torch.float32, "lr") if lr is not None else None, n, _stream()))
    return loss, grad, lr


def fipt_render_loss_masked(shading: torch.Tensor, material: torch.Tensor, observed: torch.Tensor,
                            sigma, alpha: torch.Tensor = None, lambda_d: float = 0.0,
                            tonemap: int = TONEMAP_NONE, want_grad: bool = True,
                            want_grad_alpha: bool = True, want_lr: bool = False,
                            loss_buf: torch.Tensor = None, grad: torch.Tensor = None,
                            grad_alpha: torch.Tensor = None, lr: torch.Tensor = None):
    """Emission-masked loss plus the diffuse prior.  Returns (loss_buf,
    grad [5, n], grad_alpha [n], Lr [3, n]) with None for what was not asked
    for; alpha [n] float32 GPU or None (zero)."""
    K = len(sigma)
    n = material.shape[1]
    if shading.shape[0] != 3 + 6 * K or shading.shape[1] != n:
        raise ValueError("shading must be [3 + 6K, n]")
    if material.shape[0] != 5 or observed.shape != (3, n):
        raise ValueError("material must be [5, n] and observed [3, n]")
    if alpha is not None:
        _need(alpha, (n,), "alpha")
    dev = material.device
    if loss_buf is None:
        loss_buf = torch.empty((LOSS_SLOTS,), dtype=torch.float64, device=dev)
    _need(loss_buf, (LOSS_SLOTS,), "loss_buf")
    if want_grad and grad is None:
        grad = torch.empty((5, n), dtype=torch.float32, device=dev)
    if want_grad:
        _need(grad, (5, n), "grad")
    if want_grad_alpha and grad_alpha is None:
        grad_alpha = torch.empty((n,), dtype=torch.float32, device=dev)
    if want_grad_alpha:
        _need(grad_alpha, (n,), "grad_alpha")
    if want_lr and lr is None:
        lr = torch.empty((3, n), dtype=torch.float32, device=dev)
    if want_lr:
        _need(lr, (3, n), "lr")
    sh = Shading(_dev(shading, torch.float32, "shading"), n)
    sig = _f32_array(sigma, K)
    _check(lib().fipt_render_loss_masked(
        C.byref(sh), n, K, sig, _dev(material, torch.float32, "material"), n,
        _dev(observed, torch.float32, "observed"), n,
        _dev(alpha, torch.float32, "alpha") if alpha is not None else None, int(tonemap),
        float(lambda_d), _dev(loss_buf, torch.float64, "loss_buf"),
        _dev(grad, torch.float32, "grad") if want_grad else None, n,
        _dev(grad_alpha, torch.float32, "grad_alpha") if want_grad_alpha else None,
        _dev(lr, torch.float32, "lr") if want_lr else None, n, _stream()))
    return (loss_buf, grad if want_grad else None, grad_alpha if want_grad_alpha else None,
            lr if want_lr else None)


def fipt_scale_by(x: torch.Tensor, factor: torch.Tensor, out: torch.Tensor = None):
    """out = x * factor[0] (factor: one float64 on the GPU) in a HIP kernel."""
    if out is None:
        out = torch.empty_like(x)
    _need(out, x.shape, "out")
    _need(factor, (1,), "factor")
    _check(lib().fipt_scale_by(_dev(x, torch.float32, "x"), x.numel(),
                               _dev(factor, torch.float64, "factor"),
                               _dev(out, torch.float32, "out"), _stream()))
    return out


def fipt_hbm_stream(kind: int, a: torch.Tensor, c: torch.Tensor, b: torch.Tensor = None,
                    s: float = 1.0):
    """Bandwidth probe: kind 0 copies a into c, kind 1 writes a + s b into c
    (float32 GPU tensors of equal size)."""
    n = a.numel()
    _need(c, a.shape, "c")
    if kind == 1:
        _need(b, a.shape, "b")
    _check(lib().fipt_hbm_stream(int(kind), _dev(a, torch.float32, "a"),
                                 _dev(b, torch.float32, "b") if kind == 1 else None,
                                 _dev(c, torch.float32, "c"), n, float(s), _stream()))
    return c


class FactoredLoss(torch.autograd.Function):
    """loss = sum (Gamma(Lr(material)) - Gamma(Lgt))^2 with the hand-written
    gradient of the library; differentiable in ``material`` [5, n]."""

    @staticmethod
    def forward(ctx, material, shading, observed, sigma, tonemap=TONEMAP_NONE):
        buf, grad, _ = fipt_render_loss(shading, material.detach(), observed, sigma, tonemap,
                                        want_grad=material.requires_grad)
        ctx.save_for_backward(grad if grad is not None else material.new_empty(0))
        return buf[0]

    @staticmethod
    def backward(ctx, go):
        (grad,) = ctx.saved_tensors
        g = fipt_scale_by(grad, go.reshape(1).to(torch.float64).contiguous())
        return g, None, None, None, None


class MaskedFactoredLoss(torch.autograd.Function):
    """Emission-masked loss plus diffuse prior (library gradients);
    differentiable in ``material`` [5, n] and ``alpha`` [n]."""

    @staticmethod
    def forward(ctx, material, alpha, shading, observed, sigma, tonemap=TONEMAP_NONE, lambda_d=0.0):
        buf, grad, galpha, _ = fipt_render_loss_masked(
            shading, material.detach(), observed, sigma, alpha.detach(), lambda_d, tonemap,
            want_grad=material.requires_grad, want_grad_alpha=alpha.requires_grad)
        empty = material.new_empty(0)
        ctx.save_for_backward(grad if grad is not None else empty,
                              galpha if galpha is not None else empty)
        return buf[0]

    @staticmethod
    def backward(ctx, go):
        grad, galpha = ctx.saved_tensors
        f = go.reshape(1).to(torch.float64).contiguous()
        gm = fipt_scale_by(grad, f) if grad.numel() else None
        ga = fipt_scale_by(galpha, f) if galpha.numel() else None
        return gm, ga, None, None, None, None, None


# --------------------------------------------------------------------------
# trilinear material grid
# --------------------------------------------------------------------------
def fipt_grid_gather(grid: torch.Tensor, bmin, bmax, pos: torch.Tensor, out: torch.Tensor = None):
    """grid [C, R, R, R] float32 GPU (x fastest), pos [3, n] -> [C, n]."""
    if grid.dim() != 4 or not (grid.shape[1] == grid.shape[2] == grid.shape[3]):
        raise ValueError(f"grid must be [C, R, R, R], got {tuple(grid.shape)}")
    if pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError(f"pos must be [3, n], got {tuple(pos.shape)}")
    Cn, R = grid.shape[0], grid.shape[1]
    n = pos.shape[1]
    if out is None:
        out = torch.empty((Cn, n), dtype=torch.float32, device=grid.device)
    _need(out, (Cn, n), "out")
    _check(lib().fipt_grid_gather(_dev(grid, torch.float32, "grid"), Cn, R, _f32_array(bmin, 3),
                                  _f32_array(bmax, 3), _dev(pos, torch.float32, "pos"), n, n,
                                  _dev(out, torch.float32, "out"), n, _stream()))
    return out


class GridPlan:
    """Deterministic adjoint of the grid gather for a fixed point set."""

    def __init__(self, pos_host, res: int, bmin, bmax, device: int = 0):
        import numpy as np
        p = np.ascontiguousarray(pos_host, dtype=np.float32)
        self.n = int(p.shape[1])
        self.res = int(res)
        h = C.c_void_p()
        _check(lib().fipt_grid_plan_create(p.ctypes.data, self.n, self.res, _f32_array(bmin, 3),
                                           _f32_array(bmax, 3), device, C.byref(h)))
        self.handle = h

    def scatter(self, grad_points: torch.Tensor, out: torch.Tensor = None):
        if grad_points.dim() != 2 or grad_points.shape[1] < self.n:
            raise ValueError(f"grad_points must be [C, >= {self.n}], got {tuple(grad_points.shape)}")
        Cn = grad_points.shape[0]
        if out is None:
            out = torch.empty((Cn, self.res, self.res, self.res), dtype=torch.float32,
                              device=grad_points.device)
        _need(out, (Cn, self.res, self.res, self.res), "out")
        _check(lib().fipt_grid_scatter(self.handle, _dev(grad_points, torch.float32, "grad_points"),
                                       Cn, grad_points.shape[1], _dev(out, torch.float32, "out"),
                                       _stream()))
        return out

    def order(self):
        """numpy int32 [n]: the original index of each point in the plan's order."""
        import numpy as np
        out = np.empty(self.n, dtype=np.int32)
        _check(lib().fipt_grid_plan_order(self.handle, out.ctypes.data))
        return out

    def permute(self, src: torch.Tensor, out: torch.Tensor = None):
        """[planes, n] float32 (or int32) GPU in point order -> the same planes in the plan's order."""
        if src.dim() != 2 or src.shape[1] != self.n:
            raise ValueError(f"src must be [planes, {self.n}], got {tuple(src.shape)}")
        if src.dtype not in (torch.float32, torch.int32):
            raise ValueError("src must be float32 or int32")
        if out is None:
            out = torch.empty_like(src)
        _need(out, tuple(src.shape), "out")
        if out.dtype != src.dtype:
            raise ValueError("out must have src's dtype")
        _check(lib().fipt_grid_plan_permute(self.handle, _dev(src, src.dtype, "src"), src.shape[0], self.n,
                                            _dev(out, out.dtype, "out"), self.n, _stream()))
        return out

    def render_loss(self, grid: torch.Tensor, shading: torch.Tensor, observed: torch.Tensor, sigma,
                    tonemap: int = TONEMAP_NONE, loss_buf: torch.Tensor = None,
                    grad_grid: torch.Tensor = None, grad_points: torch.Tensor = None):
        """Fused material fetch + render + loss + grid adjoint for the plan's points, with
        shading [3 + 6K, n] and observed [3, n] in the plan's order.  Returns
        (loss_buf, grad_grid [5, R, R, R]); loss_buf[0] is the loss.  grad_points [5, n]
        (plan order), when given, receives the per-point material gradient."""
        K = len(sigma)
        R = self.res
        if grid.shape != (5, R, R, R):
            raise ValueError(f"grid must be [5, {R}, {R}, {R}], got {tuple(grid.shape)}")
        if shading.shape != (3 + 6 * K, self.n) or observed.shape != (3, self.n):
            raise ValueError("shading must be [3 + 6K, n] and observed [3, n]")
        dev = grid.device
        if loss_buf is None:
            loss_buf = torch.empty((LOSS_SLOTS,), dtype=torch.float64, device=dev)
        _need(loss_buf, (LOSS_SLOTS,), "loss_buf")
        if grad_grid is None:
            grad_grid = torch.empty_like(grid)
        _need(grad_grid, (5, R, R, R), "grad_grid")
        if grad_points is not None:
            _need(grad_points, (5, self.n), "grad_points")
        sh = Shading(_dev(shading, torch.float32, "shading"), self.n)
        _check(lib().fipt_grid_render_loss(
            self.handle, _dev(grid, torch.float32, "grid"), C.byref(sh), K, _f32_array(sigma, K),
            _dev(observed, torch.float32, "observed"), self.n, int(tonemap),
            _dev(loss_buf, torch.float64, "loss_buf"), _dev(grad_grid, torch.float32, "grad_grid"),
            _dev(grad_points, torch.float32, "grad_points") if grad_points is not None else None,
            self.n, _stream()))
        return loss_buf, grad_grid

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_grid_plan_destroy(self.handle)
        except Exception:
            pass


class EmissionPlan:
    """Per-triangle emission re-estimation (Eq. 13 with f = 0): the pixels
    grouped by their primary-hit triangle once (``tri_host`` [n], -1 for
    none), then ``median`` of the observations per emitter triangle."""

    def __init__(self, tri_host, n_tris: int, device: int = 0):
        import numpy as np
        t = np.ascontiguousarray(tri_host, dtype=np.int32)
        if t.ndim != 1:
            raise ValueError("tri_host must be [n]")
        self.n = int(t.shape[0])
        self.n_tris = int(n_tris)
        h = C.c_void_p()
        _check(lib().fipt_emission_plan_create(t.ctypes.data, self.n, self.n_tris, device, C.byref(h)))
        self.handle = h

    def median(self, observed: torch.Tensor, emitter: torch.Tensor, out: torch.Tensor = None):
        """observed [3, n] float32 GPU, emitter [n_tris] uint8 (or bool) GPU
        -> Le [3, n_tris] float32 GPU."""
        if observed.dim() != 2 or observed.shape[0] != 3 or observed.shape[1] != self.n:
            raise ValueError(f"observed must be [3, {self.n}], got {tuple(observed.shape)}")
        if emitter.dtype == torch.bool:
            emitter = emitter.to(torch.uint8)
        _need(emitter, (self.n_tris,), "emitter")
        if out is None:
            out = torch.empty((3, self.n_tris), dtype=torch.float32, device=observed.device)
        _need(out, (3, self.n_tris), "out")
        _check(lib().fipt_emission_median(self.handle, _dev(observed, torch.float32, "observed"), self.n,
                                          _dev(emitter, torch.uint8, "emitter"),
                                          _dev(out, torch.float32, "out"), self.n_tris, _stream()))
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_emission_plan_destroy(self.handle)
        except Exception:
            pass


class VoxelPlan:
    """Average pooling of observed pixels onto a voxel grid (the radiance
    cache of Sec. 4.2): the pixels' surface points ``pos_host`` [3, n] are
    sorted by voxel of a res^3 grid over [bmin, bmax] once; ``pool`` then
    averages observations per voxel."""

    def __init__(self, pos_host, res: int, bmin, bmax, device: int = 0):
        import numpy as np
        pos = np.ascontiguousarray(pos_host, dtype=np.float32)
        if pos.ndim != 2 or pos.shape[0] != 3:
            raise ValueError("pos_host must be [3, n]")
        self.n = int(pos.shape[1])
        self.res = int(res)
        self.bmin = [float(v) for v in bmin]
        self.bmax = [float(v) for v in bmax]
        h = C.c_void_p()
        _check(lib().fipt_voxel_plan_create(pos.ctypes.data, self.n, self.res,
                                            _f32_array(self.bmin, 3), _f32_array(self.bmax, 3),
                                            device, C.byref(h)))
        self.handle = h

    def pool(self, observed: torch.Tensor, out: torch.Tensor = None):
        """observed [3, n] float32 GPU -> cache [3, res^3] float32 GPU."""
        if observed.dim() != 2 or observed.shape[0] != 3 or observed.shape[1] != self.n:
            raise ValueError(f"observed must be [3, {self.n}], got {tuple(observed.shape)}")
        nv = self.res ** 3
        if out is None:
            out = torch.empty((3, nv), dtype=torch.float32, device=observed.device)
        _need(out, (3, nv), "out")
        _check(lib().fipt_voxel_pool(self.handle, _dev(observed, torch.float32, "observed"), self.n,
                                     _dev(out, torch.float32, "out"), nv, _stream()))
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_voxel_plan_destroy(self.handle)
        except Exception:
            pass


# hash-grid material network (Eq. 14): tables [32][2^19][2], W1, W2 [64][64], W3 [5][64]
HG_PARAMS = 32 * (1 << 19) * 2 + 64 * 64 + 64 * 64 + 5 * 64


def fipt_hashgrid_forward(params: torch.Tensor, pos: torch.Tensor, bmin, bmax,
                          out: torch.Tensor = None):
    """params [HG_PARAMS] float32 GPU, pos [3, n] -> material [5, n]."""
    _need(params, (HG_PARAMS,), "params")
    if pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError(f"pos must be [3, n], got {tuple(pos.shape)}")
    n = pos.shape[1]
    if out is None:
        out = torch.empty((5, n), dtype=torch.float32, device=pos.device)
    _need(out, (5, n), "out")
    _check(lib().fipt_hashgrid_forward(_dev(params, torch.float32, "params"),
                                       _dev(pos, torch.float32, "pos"), n, n, _f32_array(bmin, 3),
                                       _f32_array(bmax, 3), _dev(out, torch.float32, "out"), n,
                                       _stream()))
    return out


class HashGridPlan:
    """Table-gradient plan of a fixed point set for the hash-grid network's
    backward pass: per level, every (point, corner) of nonzero weight sorted
    by table slot, built on the GPU once.  Holds ``pos`` [3, n] and the box
    for the forward pass too."""

    def __init__(self, pos: torch.Tensor, bmin, bmax):
        if pos.dim() != 2 or pos.shape[0] != 3:
            raise ValueError(f"pos must be [3, n], got {tuple(pos.shape)}")
        self.pos = pos.contiguous()
        self.n = int(pos.shape[1])
        self.bmin, self.bmax = list(map(float, bmin)), list(map(float, bmax))
        h = C.c_void_p()
        _check(lib().fipt_hashgrid_plan_create(_dev(self.pos, torch.float32, "pos"), self.n, self.n,
                                               _f32_array(self.bmin, 3), _f32_array(self.bmax, 3),
                                               _stream(), C.byref(h)))
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_hashgrid_plan_destroy(self.handle)
        except Exception:
            pass


def hashgrid_workspace(n: int, device) -> torch.Tensor:
    """A workspace for the hash-grid backward pass of n points."""
    return torch.empty((int(lib().fipt_hashgrid_workspace_floats(n)),), dtype=torch.float32,
                       device=device)


def fipt_hashgrid_forward_save(params: torch.Tensor, plan: "HashGridPlan", workspace: torch.Tensor,
                               out: torch.Tensor = None):
    """The forward pass for the plan's points that also keeps their hash
    encoding in ``workspace`` for fipt_hashgrid_backward(..., saved=True)."""
    _need(params, (HG_PARAMS,), "params")
    n = plan.n
    need = int(lib().fipt_hashgrid_workspace_floats(n))
    if workspace.dim() != 1 or workspace.shape[0] < need:
        raise ValueError(f"workspace must hold at least {need} floats")
    if out is None:
        out = torch.empty((5, n), dtype=torch.float32, device=params.device)
    _need(out, (5, n), "out")
    _check(lib().fipt_hashgrid_forward_save(_dev(params, torch.float32, "params"),
                                            _dev(plan.pos, torch.float32, "pos"), n, n,
                                            _f32_array(plan.bmin, 3), _f32_array(plan.bmax, 3),
                                            _dev(out, torch.float32, "out"), n,
                                            _dev(workspace, torch.float32, "workspace"),
                                            workspace.shape[0], _stream()))
    return out


def fipt_hashgrid_backward(plan: HashGridPlan, params: torch.Tensor, grad_material: torch.Tensor,
                           grad_params: torch.Tensor = None, workspace: torch.Tensor = None,
                           saved: bool = False):
    """Adds d(sum grad_material * material) / d params, for the plan's
    points, into grad_params (zeros if None) and returns it.  With ``saved``
    the workspace holds the encoding fipt_hashgrid_forward_save left there."""
    _need(params, (HG_PARAMS,), "params")
    if saved and workspace is None:
        raise ValueError("saved needs the workspace of fipt_hashgrid_forward_save")
    n = plan.n
    _need(grad_material, (5, n), "grad_material")
    if grad_params is None:
        grad_params = torch.zeros((HG_PARAMS,), dtype=torch.float32, device=params.device)
    _need(grad_params, (HG_PARAMS,), "grad_params")
    need = int(lib().fipt_hashgrid_workspace_floats(n))
    if workspace is None:
        workspace = torch.empty((need,), dtype=torch.float32, device=params.device)
    if workspace.dim() != 1 or workspace.shape[0] < need:
        raise ValueError(f"workspace must hold at least {need} floats")
    fn = lib().fipt_hashgrid_backward_saved if saved else lib().fipt_hashgrid_backward
    _check(fn(plan.handle, _dev(params, torch.float32, "params"),
              _dev(grad_material, torch.float32, "grad_material"), n,
              _dev(grad_params, torch.float32, "grad_params"),
              _dev(workspace, torch.float32, "workspace"), workspace.shape[0], _stream()))
    return grad_params


class HashGridMaterial(torch.autograd.Function):
    """material [5, n] = Sigmoid(MLP(hash encoding(plan.pos))); differentiable
    in ``params`` through the library's backward pass."""

    @staticmethod
    def forward(ctx, params, plan):
        ctx.save_for_backward(params)
        ctx.plan = plan
        # the encoding is kept for the backward pass (256 B per point)
        ctx.ws = hashgrid_workspace(plan.n, params.device)
        return fipt_hashgrid_forward_save(params.detach(), plan, ctx.ws)

    @staticmethod
    def backward(ctx, g):
        (params,) = ctx.saved_tensors
        gp = fipt_hashgrid_backward(ctx.plan, params.detach(), g.contiguous(), workspace=ctx.ws,
                                    saved=True)
        ctx.ws = None
        return gp, None


class GridGather(torch.autograd.Function):
    """Per-point values of a trilinear grid, differentiable in the grid."""

    @staticmethod
    def forward(ctx, grid, plan: GridPlan, bmin, bmax, pos):
        ctx.plan = plan
        return fipt_grid_gather(grid.detach(), bmin, bmax, pos)

    @staticmethod
    def backward(ctx, go):
        return ctx.plan.scatter(go.contiguous()), None, None, None, None


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------
@dataclass
class Result:
    shading: torch.Tensor
    t_submit_us: int
    t_admit_us: int
    t_done_us: int


class Server:
    """Continuous-batching bake server (fipt_server_*)."""

    def __init__(self, device: int = 0, pool_bytes: int = 4 << 30, max_inflight: int = 64,
                 samples_per_launch: int = 1 << 26):
        h = C.c_void_p()
        _check(lib().fipt_server_create(device, int(pool_bytes), int(max_inflight),
                                        int(samples_per_launch), C.byref(h)))
        self.handle = h
        self.device = device
        self._keep = {}

    def submit(self, scene: Scene, planes: torch.Tensor, tri: torch.Tensor, spp_d, spp_s, sigma,
               seed, ray_eps=1e-4, offset: int = 0, count: int = None) -> int:
        """Queue the bake of points [offset, offset + count) of (planes, tri)."""
        n_all = planes.shape[1]
        count = n_all - offset if count is None else int(count)
        pts = Points(_dev(planes, torch.float32, "planes") + 4 * offset,
                     _dev(tri, torch.int32, "tri") + 4 * offset, count, n_all)
        par = make_params(spp_d, spp_s, sigma, seed, ray_eps)
        t = C.c_uint64()
        _check(lib().fipt_server_submit(self.handle, scene.handle, C.byref(pts), C.byref(par),
                                        C.byref(t)))
        self._keep[t.value] = (planes, tri, len(sigma), count)
        return t.value

    def poll(self, ticket: int) -> bool:
        return _check(lib().fipt_server_poll(self.handle, ticket), allow=(EAGAIN,)) == OK

    def wait(self, ticket: int, timeout_s: float = -1.0) -> bool:
        us = -1 if timeout_s < 0 else int(timeout_s * 1e6)
        return _check(lib().fipt_server_wait(self.handle, ticket, us), allow=(EAGAIN,)) == OK

    def result(self, ticket: int, copy: bool = True) -> Result:
        sh = Shading()
        ts, ta, td = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().fipt_server_result(self.handle, ticket, C.byref(sh), C.byref(ts), C.byref(ta),
                                        C.byref(td)))
        _, _, K, count = self._keep[ticket]
        P = 3 + 6 * K
        t = None
        if copy:
            # view the pool memory through a DLPack-free wrapper: copy on the
            # server's results by a device-to-device memcpy into a tensor
            t = torch.empty((P, count), dtype=torch.float32, device=torch.device("cuda", self.device))
            torch.cuda.synchronize(self.device)
            hip = _hip()
            rc = hip.hipMemcpy(C.c_void_p(t.data_ptr()), C.c_void_p(sh.planes),
                               C.c_size_t(4 * P * count), 3)
            if rc != 0:
                raise FiptError(EHIP, f"hipMemcpy failed ({rc})")
        return Result(t, ts.value, ta.value, td.value)

    def release(self, ticket: int):
        _check(lib().fipt_server_release(self.handle, ticket))
        self._keep.pop(ticket, None)

    def cancel(self, ticket: int):
        _check(lib().fipt_server_cancel(self.handle, ticket))

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(lib().fipt_server_stats_get(self.handle, C.byref(s)))
        return s

    def destroy(self):
        if self.handle:
            _check(lib().fipt_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.fipt_server_destroy(self.handle)
        except Exception:
            pass


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = C.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.restype = C.c_int
        _hip_lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hip_lib
