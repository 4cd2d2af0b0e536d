"""Python side of the C oracle: shading points (camera rays through pixel
centres) and the Monte Carlo bake of the factorized shading terms (Eq. 6 with
the Fresnel split of Eq. 7 and the stage-1 radiance query of Eq. 9), in
double precision with brute-force ray casting.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

WEAK_FURNACE = 1
EOVERFLOW = -2


class CandidateOverflow(RuntimeError):
    """A ray met more candidate outcomes than the C oracle keeps (256): its
    envelope would be incomplete, so the result is refused."""


def _checked(rc: int, what: str) -> int:
    if rc == EOVERFLOW:
        raise CandidateOverflow(f"{what}: a ray met more than 256 candidate outcomes")
    return rc


_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    stale = (not os.path.exists(_build.LIB)
             or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC))
    if stale:
        _build.build()
    L = C.CDLL(_build.LIB)
    L.orc_scene_new.restype = C.c_void_p
    L.orc_scene_new.argtypes = [_f32p, C.c_int64, _i32p, C.c_int64, C.c_int,
                                _f32p, _f32p, C.c_double, C.c_double]
    L.orc_scene_free.argtypes = [C.c_void_p]
    L.orc_scene_set_voxel.restype = C.c_int
    L.orc_scene_set_voxel.argtypes = [C.c_void_p, _f32p, C.c_int, _f64p, _f64p]
    L.orc_philox.argtypes = [_u32p, _u32p, _u32p, C.c_int64]
    L.orc_lobe_uniforms.argtypes = [C.c_uint64, _i64p, _i32p, _i32p, _i32p, C.c_int64,
                                    _f64p, _f64p]
    L.orc_frame.argtypes = [_f64p, _f64p, _f64p]
    L.orc_sample_cosine.argtypes = [C.c_double, C.c_double, _f64p]
    L.orc_sample_ggx.argtypes = [C.c_double, C.c_double, C.c_double, _f64p]
    L.orc_ggx_D.restype = C.c_double
    L.orc_ggx_D.argtypes = [C.c_double, C.c_double]
    L.orc_ggx_G1.restype = C.c_double
    L.orc_ggx_G1.argtypes = [C.c_double, C.c_double]
    L.orc_cast.restype = C.c_int
    L.orc_trace_radiance.restype = C.c_int
    L.orc_cast.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int64, _i32p, _f64p,
                           _f64p, _i32p]
    L.orc_trace_radiance.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int64, _f64p]
    L.orc_primary.restype = C.c_int
    L.orc_primary.argtypes = [C.c_void_p, _f32p, _i32p, C.c_int, _i64p, C.c_int64,
                              _f64p, _i32p, _i32p, C.c_int]
    L.orc_bake.restype = C.c_int
    L.orc_bake.argtypes = [C.c_void_p, _f32p, _i32p, C.c_int64, _i64p, C.c_int64,
                           C.c_int, C.c_int, C.c_int, _f64p, C.c_uint64,
                           C.c_double, C.c_int, C.c_int, _f64p, _f64p, _f64p,
                           _f64p, C.POINTER(C.c_int64)]
    L.orc_quadrature.restype = C.c_int
    L.orc_quadrature.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, C.c_int,
                                 C.c_double, C.c_int, C.c_int, C.c_double, _f64p]
    L.orc_max_threads.restype = C.c_int
    L.orc_refine.restype = C.c_int
    L.orc_refine.argtypes = [C.c_void_p, _f32p, _i32p, C.c_int64, _i64p, C.c_int64,
                             C.c_int, C.c_int, C.c_int, _f64p, C.c_uint64, C.c_double,
                             _f32p, C.c_int, _f64p, _f64p, C.c_double, C.c_int, C.c_int,
                             C.c_int, _f64p, _f64p, _f64p, _f64p, C.POINTER(C.c_int64)]
    L.orc_refine_quadrature.restype = C.c_int
    L.orc_refine_quadrature.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, C.c_int, C.c_double,
                                        _f32p, C.c_int, _f64p, _f64p, C.c_double, C.c_int,
                                        C.c_int, C.c_int, C.c_int, C.c_double, _f64p]
    L.orc_brdf.argtypes = [_f64p, _f64p, _f64p, _f64p, C.c_double, C.c_double, _f64p]
    L.orc_material_at.argtypes = [_f32p, C.c_int, _f64p, _f64p, _f64p, C.c_int64, _f64p]
    L.orc_brdf_pdf.restype = C.c_double
    L.orc_brdf_pdf.argtypes = [_f64p, _f64p, _f64p, C.c_double]
    _lib = L
    return L


def max_threads() -> int:
    return int(lib().orc_max_threads())


class OracleScene:
    """Double-precision copy of a scene.  ``tol_rel`` sets the ambiguity band:
    a hit within tol_rel * (1 + t) of a triangle edge, or within that
    distance of a nearer surface, is one single-precision arithmetic may
    resolve either way."""

    def __init__(self, scene, tol_rel: float = 1e-5):
        self.scene = scene
        verts = np.ascontiguousarray(scene.verts, dtype=np.float32)
        tris = np.ascontiguousarray(scene.tris, dtype=np.int32)
        cache = np.ascontiguousarray(scene.cache, dtype=np.float32)
        emission = np.ascontiguousarray(scene.emission, dtype=np.float32)
        kind = 1 if scene.cache_kind == "vertex" else 0
        ext = verts.max(0).astype(np.float64) - verts.min(0).astype(np.float64)
        max_t = float(np.linalg.norm(ext)) * 2.0 + 1.0
        self._keep = (verts, tris, cache, emission)
        self.handle = lib().orc_scene_new(verts, len(verts), tris, len(tris), kind,
                                          cache, emission, tol_rel, max_t)

    def set_voxel_cache(self, cache, res: int, lo, hi):
        """Use a voxel grid cache [3, res^3] (x fastest) over the box
        [lo, hi] instead of the scene's own cache: a hit reads the voxel
        that contains it (Sec. 4.2, nearest-voxel query)."""
        c = np.ascontiguousarray(cache, dtype=np.float32).reshape(3, -1)
        if c.shape[1] != res ** 3:
            raise ValueError("cache must be [3, res^3]")
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        if lib().orc_scene_set_voxel(self.handle, c, int(res), lo, hi) != 0:
            raise ValueError("bad voxel grid")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.orc_scene_free(self.handle)
            self.handle = None


# -------------------------------------------------------------------------
# primitives (test hooks)
# -------------------------------------------------------------------------
def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().orc_philox(ctr, key, out, len(ctr))
    return out


def lobe_uniforms(seed: int, p, lobe, s, n):
    """(xi1, xi2) of sample s of n for lobe `lobe` of point p (arrays,
    broadcast): Philox4x32-10 on the counter (p low, p high, lobe, s) under
    key `seed`, stratified along the Z-order curve (``sample_uniforms`` in
    the C oracle)."""
    p, lobe, s, n = np.broadcast_arrays(np.asarray(p, np.int64), np.asarray(lobe, np.int32),
                                        np.asarray(s, np.int32), np.asarray(n, np.int32))
    p = np.ascontiguousarray(p.ravel())
    lobe = np.ascontiguousarray(lobe.ravel())
    s = np.ascontiguousarray(s.ravel())
    n = np.ascontiguousarray(n.ravel())
    if np.any(n < 1) or np.any(s < 0) or np.any(s >= n):
        raise ValueError("need 0 <= s < n")
    xi1 = np.empty(len(p), np.float64)
    xi2 = np.empty(len(p), np.float64)
    lib().orc_lobe_uniforms(C.c_uint64(seed), p, lobe, s, n, len(p), xi1, xi2)
    return xi1, xi2


def frame(n):
    n = np.ascontiguousarray(n, dtype=np.float64)
    t = np.zeros(3)
    b = np.zeros(3)
    lib().orc_frame(n, t, b)
    return t, b


def sample_cosine(xi1, xi2):
    out = np.zeros(3)
    lib().orc_sample_cosine(float(xi1), float(xi2), out)
    return out


def sample_ggx(alpha, xi1, xi2):
    out = np.zeros(3)
    lib().orc_sample_ggx(float(alpha), float(xi1), float(xi2), out)
    return out


def ggx_D(alpha, cos_m):
    return lib().orc_ggx_D(float(alpha), float(cos_m))


def ggx_G1(alpha, cos_v):
    return lib().orc_ggx_G1(float(alpha), float(cos_v))


def cast(osc: OracleScene, o: np.ndarray, d: np.ndarray):
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = len(o)
    tri = np.zeros(n, np.int32)
    t = np.zeros(n)
    b = np.zeros((n, 2))
    nc = np.zeros(n, np.int32)
    _checked(lib().orc_cast(osc.handle, o, d, n, tri, t, b, nc), "cast")
    return tri, t, b, nc


def trace_radiance(osc: OracleScene, o: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Radiance arriving at o from direction d: cache plus emission at the
    nearest hit, zero on a miss.  Returns float64 [n, 3]."""
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    R = np.zeros((len(o), 3))
    _checked(lib().orc_trace_radiance(osc.handle, o, d, len(o), R), "trace_radiance")
    return R


# -------------------------------------------------------------------------
# shading points
# -------------------------------------------------------------------------
def primary(osc: OracleScene, idx=None, threads: int = 0):
    """Camera ray through each listed pixel centre -> closest hit.
    Returns dict(points=[9, n] float64 (x, n, wo), tri=int32[n],
    n_outcomes=int32[n] (1 = unambiguous))."""
    sc = osc.scene
    cams = np.ascontiguousarray(sc.camera_array(), dtype=np.float32)
    sizes = np.ascontiguousarray(sc.camera_sizes(), dtype=np.int32)
    if idx is None:
        idx = np.arange(sc.n_points, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    out = np.zeros((9, n), np.float64)
    tri = np.zeros(n, np.int32)
    amb = np.zeros(n, np.int32)
    rc = _checked(lib().orc_primary(osc.handle, cams, sizes, len(cams), idx, n, out, tri,
                                    amb, int(threads)), "primary")
    if rc != 0:
        raise ValueError("pixel index out of range")
    return dict(points=out, tri=tri, n_outcomes=amb)


def points_f32(prim: dict):
    """Round the oracle's shading points to the single-precision SoA planes
    the bake consumes."""
    return (np.ascontiguousarray(prim["points"].astype(np.float32)),
            np.ascontiguousarray(prim["tri"].astype(np.int32)))


# -------------------------------------------------------------------------
# the bake
# -------------------------------------------------------------------------
def bake(osc: OracleScene, pts: np.ndarray, tri: np.ndarray, idx=None,
         spp_d: int = 64, spp_s: int = 64, sigma=None, seed: int = 0,
         eps: float = 1e-4, flags: int = 0, threads: int = 0):
    """Monte Carlo bake of the listed points.

    pts: float32 [9, stride] planes px py pz nx ny nz ox oy oz; tri int32
    [stride].  Returns dict(mean, lo, hi, sq) each float64 [3 + 6K, n] in
    plane order Ld(3), Ls0 per level (3 each), Ls1 per level (3 each), and
    n_ambiguous (number of ambiguous samples)."""
    if sigma is None:
        sigma = osc.scene.sigma
    # the library receives its roughness levels in single precision; the
    # oracle promotes exactly those values
    sigma = np.ascontiguousarray(np.asarray(sigma, dtype=np.float32), dtype=np.float64)
    K = len(sigma)
    pts = np.ascontiguousarray(pts, dtype=np.float32)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    stride = pts.shape[1]
    if idx is None:
        idx = np.arange(stride, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    P = 3 + 6 * K
    mean = np.zeros((P, n))
    lo = np.zeros((P, n))
    hi = np.zeros((P, n))
    sq = np.zeros((P, n))
    namb = C.c_int64(0)
    _checked(lib().orc_bake(osc.handle, pts, tri, stride, idx, n, int(spp_d), int(spp_s), K,
                            sigma, C.c_uint64(int(seed)), float(eps), int(flags), int(threads),
                            mean, lo, hi, sq, C.byref(namb)), "bake")
    return dict(mean=mean, lo=lo, hi=hi, sq=sq, n_ambiguous=int(namb.value))


def std_error(res: dict, spp_d: int, spp_s: int) -> np.ndarray:
    """Standard error of each Monte Carlo mean from the per-sample second
    moment."""
    P = res["mean"].shape[0]
    cnt = np.array([spp_d] * 3 + [spp_s] * (P - 3), dtype=np.float64)[:, None]
    var_of_mean = res["sq"] - res["mean"] ** 2 / cnt
    return np.sqrt(np.maximum(var_of_mean, 0.0) * cnt / np.maximum(cnt - 1, 1))


def quadrature(osc: OracleScene, x, n, wo, lobe: int, sigma: float = 0.0,
               n_theta: int = 512, n_phi: int = 512, eps: float = 1e-4):
    """Deterministic quadrature of one shading integral at one point.
    lobe < 0: Ld (returns 3 values); lobe >= 0: (Ls0, Ls1) at roughness
    ``sigma`` (returns 6 values)."""
    out = np.zeros(6)
    _checked(lib().orc_quadrature(osc.handle, np.ascontiguousarray(x, np.float64),
                         np.ascontiguousarray(n, np.float64),
                         np.ascontiguousarray(wo, np.float64), int(lobe),
                         float(sigma), int(n_theta), int(n_phi), float(eps), out), "quadrature")
    return out[:3] if lobe < 0 else out


# -------------------------------------------------------------------------
# stage-3 path-traced refinement (Sec. 4.3, Eq. 10 and 11)
# -------------------------------------------------------------------------
REFINE_BSDF_ONLY = 1


def _grid_args(grid, lo, hi):
    g = np.ascontiguousarray(grid, dtype=np.float32)
    res = g.shape[-1]
    if g.shape != (5, res, res, res):
        raise ValueError("material grid must be [5, R, R, R]")
    return (g.reshape(-1), int(res), np.ascontiguousarray(lo, dtype=np.float64),
            np.ascontiguousarray(hi, dtype=np.float64))


def refine(osc: OracleScene, pts: np.ndarray, tri: np.ndarray, grid, grid_lo, grid_hi, idx=None,
           spp_d: int = 64, spp_s: int = 64, sigma=None, seed: int = 0, eps: float = 1e-4,
           sigma_diffuse: float = 0.6, max_vertices: int = 8, flags: int = 0, threads: int = 0):
    """Refined shading terms (Eq. 10 / 11) of the listed points, laid out
    as ``bake``'s result; ``grid`` [5, R, R, R] is the current material
    (a_r, a_g, a_b, sigma, m) over the box [grid_lo, grid_hi]."""
    if sigma is None:
        sigma = osc.scene.sigma
    sigma = np.ascontiguousarray(np.asarray(sigma, dtype=np.float32), dtype=np.float64)
    K = len(sigma)
    pts = np.ascontiguousarray(pts, dtype=np.float32)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    stride = pts.shape[1]
    if idx is None:
        idx = np.arange(stride, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    P = 3 + 6 * K
    mean, lo, hi, sq = (np.zeros((P, n)) for _ in range(4))
    namb = C.c_int64(0)
    g, res, glo, ghi = _grid_args(grid, grid_lo, grid_hi)
    rc = lib().orc_refine(osc.handle, pts, tri, stride, idx, n, int(spp_d), int(spp_s), K, sigma,
                          C.c_uint64(int(seed)), float(eps), g, res, glo, ghi, float(sigma_diffuse),
                          int(max_vertices), int(flags), int(threads), mean, lo, hi, sq,
                          C.byref(namb))
    if rc == -1:
        raise ValueError("refine: voxel cache, grid resolution below 2 or max_vertices outside [1, 16]")
    _checked(rc, "refine")
    return dict(mean=mean, lo=lo, hi=hi, sq=sq, n_ambiguous=int(namb.value))


def refine_quadrature(osc: OracleScene, x, n, wo, lobe: int, grid, grid_lo, grid_hi,
                      sigma: float = 0.0, sigma_diffuse: float = 0.6, n_theta: int = 128,
                      n_phi: int = 256, n_theta2: int = 64, n_phi2: int = 128, eps: float = 1e-4):
    """Deterministic nested quadrature of one refined shading integral for a
    scene whose paths all end by their second vertex.  Returns (values
    (3 for Ld, 6 for Ls0 and Ls1 at roughness sigma), weight of directions
    that went deeper)."""
    out = np.zeros(7)
    g, res, glo, ghi = _grid_args(grid, grid_lo, grid_hi)
    _checked(lib().orc_refine_quadrature(osc.handle, np.ascontiguousarray(x, np.float64),
                                         np.ascontiguousarray(n, np.float64),
                                         np.ascontiguousarray(wo, np.float64), int(lobe),
                                         float(sigma), g, res, glo, ghi, float(sigma_diffuse),
                                         int(n_theta), int(n_phi), int(n_theta2), int(n_phi2),
                                         float(eps), out), "refine_quadrature")
    return (out[:3] if lobe < 0 else out[:6]), out[6]


def brdf(n, wo, wi, a, sigma, m):
    """f of Eq. 1 with the cosine (RGB), as the refinement evaluates it."""
    out = np.zeros(3)
    lib().orc_brdf(*(np.ascontiguousarray(v, np.float64) for v in (n, wo, wi, a)), float(sigma),
                   float(m), out)
    return out


def brdf_pdf(n, wo, wi, sigma):
    """Density (per solid angle) of the refinement's BRDF sampling."""
    return lib().orc_brdf_pdf(*(np.ascontiguousarray(v, np.float64) for v in (n, wo, wi)),
                              float(sigma))


def material_at(grid, grid_lo, grid_hi, x):
    """The refinement's material lookup (trilinear, clamped) at points
    x [n, 3]; returns [n, 5]."""
    g, res, glo, ghi = _grid_args(grid, grid_lo, grid_hi)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((len(x), 5))
    lib().orc_material_at(g, res, glo, ghi, x, len(x), out)
    return out
