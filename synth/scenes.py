"""Seeded synthetic scenes shaped like the paper's indoor workloads.

The paper evaluates on indoor rooms with ceiling lamps, a window and small
emitters, with high-dynamic-range emission far brighter than reflected light
(Sec. 5 and supplementary capture protocol).  Its scenes and captures are not
available, so these generators stand in for them:

* ``tiny_box``      a closed unit cube, 20 triangles, one ceiling emitter;
* ``room``          a 6 x 5 x 3 m room with tessellated walls, 40 boxes and two
                    icospheres (about 190k triangles), 3 ceiling lamps and a
                    window, per-vertex radiance cache;
* ``serving_rooms`` eight rooms from 20k to 2M triangles;
* ``large_room``    a 2M-triangle room with 8 emitters and 1M shading points.

Camera placement follows the paper's capture protocol (supplementary,
real-scene capture): start facing the room centre, yaw offset in
[-60, 60] degrees, pitch in [-45, 45] degrees, no roll, height in
[0.5, 2.5] m.

Every generator uses numpy PCG64 with a fixed seed; nothing here performs
any sampling, ray casting or shading.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Roughness levels of the specular shading tables (the paper tabulates six
# levels, Eq. 8; this grid starts at 0.02 instead of 0 so every level is a
# proper GGX lobe).
SIGMA_GRID = (0.02, 0.1, 0.25, 0.5, 0.75, 1.0)


@dataclass
class Camera:
    pos: tuple
    fwd: tuple
    up: tuple
    vfov_deg: float
    width: int
    height: int

    def as_row(self) -> list:
        return [*self.pos, *self.fwd, *self.up, self.vfov_deg]


@dataclass
class Scene:
    name: str
    verts: np.ndarray          # float32 [V, 3]
    tris: np.ndarray           # int32 [T, 3]
    cache_kind: str            # "triangle" or "vertex"
    cache: np.ndarray          # float32 [3, T] or [3, V]
    emission: np.ndarray       # float32 [3, T]
    cameras: list = field(default_factory=list)
    spp: int = 64
    sigma: tuple = SIGMA_GRID
    seed: int = 0              # Philox key of the bake
    bmin: np.ndarray = None    # float32 [3] scene bounds (material grid frame)
    bmax: np.ndarray = None

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_points(self) -> int:
        return int(sum(c.width * c.height for c in self.cameras))

    def camera_array(self) -> np.ndarray:
        """float32 [n_cams, 10]: pos(3) fwd(3) up(3) vfov_deg; sizes separate."""
        return np.array([c.as_row() for c in self.cameras], dtype=np.float32)

    def camera_sizes(self) -> np.ndarray:
        return np.array([[c.width, c.height] for c in self.cameras], dtype=np.int32)


# --------------------------------------------------------------------------
# mesh assembly helpers
# --------------------------------------------------------------------------
class _Mesh:
    def __init__(self):
        self.v = []
        self.t = []
        self.cell_centre = []   # per triangle: centre of the quad cell it came from
        self.tag = []           # per triangle: surface tag
        self.nv = 0

    def add(self, verts, tris, centres, tag):
        verts = np.asarray(verts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        self.v.append(verts)
        self.t.append(tris + self.nv)
        self.cell_centre.append(np.asarray(centres, dtype=np.float64))
        self.tag.append(np.full(len(tris), tag, dtype=np.int32))
        self.nv += len(verts)

    def finish(self):
        v = np.concatenate(self.v).astype(np.float32)
        t = np.concatenate(self.t).astype(np.int32)
        c = np.concatenate(self.cell_centre)
        g = np.concatenate(self.tag)
        return v, t, c, g


def _grid_quad(origin, du, dv, nu, nv):
    """Rectangle origin + s*du + r*dv, s, r in [0, 1], split into nu x nv
    cells, two triangles per cell, vertices shared inside the rectangle."""
    origin = np.asarray(origin, dtype=np.float64)
    du = np.asarray(du, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    i = np.arange(nu + 1, dtype=np.float64) / nu
    j = np.arange(nv + 1, dtype=np.float64) / nv
    verts = origin[None, None, :] + i[:, None, None] * du + j[None, :, None] * dv
    verts = verts.reshape(-1, 3)
    ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    v00 = ii * (nv + 1) + jj
    v10 = (ii + 1) * (nv + 1) + jj
    v11 = (ii + 1) * (nv + 1) + jj + 1
    v01 = ii * (nv + 1) + jj + 1
    tris = np.empty((2 * len(ii), 3), dtype=np.int64)
    tris[0::2] = np.stack([v00, v10, v11], axis=1)
    tris[1::2] = np.stack([v00, v11, v01], axis=1)
    cu = (ii + 0.5) / nu
    cv = (jj + 0.5) / nv
    centres = origin[None, :] + cu[:, None] * du + cv[:, None] * dv
    centres = np.repeat(centres, 2, axis=0)
    return verts, tris, centres


# Regular icosahedron: 12 vertices (0, +-1, +-phi) and cyclic permutations,
# 20 faces.  Subdivision splits each face in four and projects the new
# vertices onto the sphere.
_PHI = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = np.array([
    (-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
    (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
    (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1),
], dtype=np.float64)
_ICO_F = np.array([
    (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
    (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
    (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
    (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
], dtype=np.int64)


def icosphere(level: int):
    v = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    f = _ICO_F.copy()
    for _ in range(level):
        e = np.stack([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=1).reshape(-1, 2)
        e = np.sort(e, axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = v[uniq[:, 0]] + v[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(v)
        v = np.concatenate([v, mid])
        m = (inv + base).reshape(-1, 3)   # midpoints of (a,b), (b,c), (c,a)
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
        f = np.concatenate([
            np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
            np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)])
    return v, f


def _box_faces(lo, hi, s):
    """Five faces (no bottom: boxes rest on the floor) of an axis-aligned box,
    each split into s x s cells."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    faces = [
        ((x0, y0, z1), (x1 - x0, 0, 0), (0, y1 - y0, 0)),   # top
        ((x0, y0, z0), (x1 - x0, 0, 0), (0, 0, z1 - z0)),   # -y side
        ((x0, y1, z0), (x1 - x0, 0, 0), (0, 0, z1 - z0)),   # +y side
        ((x0, y0, z0), (0, y1 - y0, 0), (0, 0, z1 - z0)),   # -x side
        ((x1, y0, z0), (0, y1 - y0, 0), (0, 0, z1 - z0)),   # +x side
    ]
    return [_grid_quad(o, du, dv, s, s) for o, du, dv in faces]


# --------------------------------------------------------------------------
# config 1: tiny closed box
# --------------------------------------------------------------------------
def tiny_box(seed: int = 1001) -> Scene:
    """Unit cube [0,1]^3, z up, closed: floor, four walls, and a ceiling made
    of four frame quads around a dyadic hole [0.375, 0.625]^2 filled by the
    emitter quad.  Ten quads, twenty triangles, every coordinate exact in
    binary.  Per-triangle radiance cache U[0,1]^3, emitter radiance 10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = 0.375, 0.625
    quads = [
        ((0, 0, 0), (1, 0, 0), (0, 1, 0)),          # floor
        ((0, 0, 0), (0, 1, 0), (0, 0, 1)),          # x = 0
        ((1, 0, 0), (0, 1, 0), (0, 0, 1)),          # x = 1
        ((0, 0, 0), (1, 0, 0), (0, 0, 1)),          # y = 0
        ((0, 1, 0), (1, 0, 0), (0, 0, 1)),          # y = 1
        ((0, 0, 1), (1, 0, 0), (0, a, 0)),          # ceiling frame y < a
        ((0, b, 1), (1, 0, 0), (0, 1 - b, 0)),      # ceiling frame y > b
        ((0, a, 1), (a, 0, 0), (0, b - a, 0)),      # ceiling frame x < a
        ((b, a, 1), (1 - b, 0, 0), (0, b - a, 0)),  # ceiling frame x > b
        ((a, a, 1), (b - a, 0, 0), (0, b - a, 0)),  # emitter
    ]
    mesh = _Mesh()
    for q, (o, du, dv) in enumerate(quads):
        v, t, c = _grid_quad(o, du, dv, 1, 1)
        mesh.add(v, t, c, q)
    verts, tris, _, tag = mesh.finish()
    T = len(tris)
    cache = rng.uniform(0.0, 1.0, size=(3, T)).astype(np.float32)
    emission = np.zeros((3, T), dtype=np.float32)
    emission[:, tag == 9] = 10.0
    cam = Camera(pos=(0.5, 0.05, 0.5), fwd=(0.0, 1.0, 0.0), up=(0.0, 0.0, 1.0),
                 vfov_deg=60.0, width=64, height=64)
    return Scene(name="tiny_box", verts=verts, tris=tris, cache_kind="triangle",
                 cache=cache, emission=emission, cameras=[cam], spp=64,
                 sigma=SIGMA_GRID, seed=2001,
                 bmin=np.zeros(3, np.float32), bmax=np.ones(3, np.float32))


# --------------------------------------------------------------------------
# configs 2, 4, 5: synthetic rooms
# --------------------------------------------------------------------------
ROOM = (6.0, 5.0, 3.0)


def _room_mesh(rng, wall_cell, sphere_level, box_sub, n_boxes=40, n_spheres=2):
    W, D, H = ROOM
    mesh = _Mesh()
    nx, ny, nz = (int(round(W / wall_cell)), int(round(D / wall_cell)),
                  int(round(H / wall_cell)))
    walls = [
        ("floor", (0, 0, 0), (W, 0, 0), (0, D, 0), nx, ny),
        ("ceiling", (0, 0, H), (W, 0, 0), (0, D, 0), nx, ny),
        ("wall_y0", (0, 0, 0), (W, 0, 0), (0, 0, H), nx, nz),
        ("wall_y1", (0, D, 0), (W, 0, 0), (0, 0, H), nx, nz),
        ("wall_x0", (0, 0, 0), (0, D, 0), (0, 0, H), ny, nz),
        ("wall_x1", (W, 0, 0), (0, D, 0), (0, 0, H), ny, nz),
    ]
    for tag, (name, o, du, dv, nu, nv) in enumerate(walls):
        v, t, c = _grid_quad(o, du, dv, nu, nv)
        mesh.add(v, t, c, tag)
    boxes = []
    for _ in range(n_boxes):
        sx, sy = rng.uniform(0.2, 1.5, size=2)
        sz = rng.uniform(0.2, 2.0)
        x0 = rng.uniform(0.1, W - sx - 0.1)
        y0 = rng.uniform(0.1, D - sy - 0.1)
        lo, hi = (x0, y0, 0.0), (x0 + sx, y0 + sy, sz)
        boxes.append((lo, hi))
        for v, t, c in _box_faces(lo, hi, box_sub):
            mesh.add(v, t, c, 10)
    spheres = []
    sv, sf = icosphere(sphere_level)
    for _ in range(n_spheres):
        r = rng.uniform(0.3, 0.6)
        cx = rng.uniform(r + 0.2, W - r - 0.2)
        cy = rng.uniform(r + 0.2, D - r - 0.2)
        cz = rng.uniform(r + 0.1, H - r - 0.3)
        spheres.append(((cx, cy, cz), r))
        centre = np.array([cx, cy, cz])
        mesh.add(sv * r + centre, sf, np.repeat(centre[None], len(sf), 0), 11)
    verts, tris, centres, tag = mesh.finish()
    return verts, tris, centres, tag, boxes, spheres


def _mark_emitters(rng, centres, tag, n_ceiling, n_window):
    """Emitters are tessellation cells marked emissive: rectangles on the
    ceiling and window rectangles on walls.  Grey radiance log-uniform in
    [1, 50]."""
    W, D, H = ROOM
    T = len(tag)
    emission = np.zeros((3, T), dtype=np.float32)
    for _ in range(n_ceiling):
        sx, sy = rng.uniform(0.6, 1.6), rng.uniform(0.3, 0.8)
        x0, y0 = rng.uniform(0.3, W - sx - 0.3), rng.uniform(0.3, D - sy - 0.3)
        L = math.exp(rng.uniform(math.log(1.0), math.log(50.0)))
        c = centres
        sel = ((tag == 1) & (c[:, 0] > x0) & (c[:, 0] < x0 + sx)
               & (c[:, 1] > y0) & (c[:, 1] < y0 + sy))
        emission[:, sel] = L
    for w in range(n_window):
        wall = [2, 3, 4, 5][(w * 3 + int(rng.integers(0, 4))) % 4]
        span = W if wall in (2, 3) else D
        sw, sh = rng.uniform(1.0, 2.0), rng.uniform(0.8, 1.4)
        s0 = rng.uniform(0.3, span - sw - 0.3)
        z0 = rng.uniform(0.8, 1.0)
        L = math.exp(rng.uniform(math.log(1.0), math.log(50.0)))
        c = centres
        along = c[:, 0] if wall in (2, 3) else c[:, 1]
        sel = ((tag == wall) & (along > s0) & (along < s0 + sw)
               & (c[:, 2] > z0) & (c[:, 2] < z0 + sh))
        emission[:, sel] = L
    return emission


def _room_cameras(rng, n, width, height, boxes, spheres):
    W, D, H = ROOM
    cams = []
    while len(cams) < n:
        p = np.array([rng.uniform(0.3, W - 0.3), rng.uniform(0.3, D - 0.3),
                      rng.uniform(0.5, 2.5)])
        yaw_off = math.radians(rng.uniform(-60.0, 60.0))
        pitch = math.radians(rng.uniform(-45.0, 45.0))
        inside = False
        for lo, hi in boxes:
            if all(lo[k] - 0.05 < p[k] < hi[k] + 0.05 for k in range(3)):
                inside = True
        for c, r in spheres:
            if np.linalg.norm(p - np.array(c)) < r + 0.05:
                inside = True
        if inside:
            continue
        to_c = np.array([W / 2, D / 2]) - p[:2]
        yaw = math.atan2(to_c[1], to_c[0]) + yaw_off
        fwd = (math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
               math.sin(pitch))
        cams.append(Camera(pos=tuple(float(x) for x in p), fwd=fwd,
                           up=(0.0, 0.0, 1.0), vfov_deg=60.0,
                           width=width, height=height))
    return cams


def _room_scene(name, seed, wall_cell, sphere_level, box_sub, n_cams, width,
                height, spp, n_ceiling, n_window, bake_seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    verts, tris, centres, tag, boxes, spheres = _room_mesh(
        rng, wall_cell, sphere_level, box_sub)
    emission = _mark_emitters(rng, centres, tag, n_ceiling, n_window)
    cache = rng.uniform(0.0, 2.0, size=(3, len(verts))).astype(np.float32)
    cams = _room_cameras(rng, n_cams, width, height, boxes, spheres)
    return Scene(name=name, verts=verts, tris=tris, cache_kind="vertex",
                 cache=cache, emission=emission, cameras=cams, spp=spp,
                 sigma=SIGMA_GRID, seed=bake_seed,
                 bmin=np.zeros(3, np.float32),
                 bmax=np.array(ROOM, dtype=np.float32))


def room(seed: int = 1002, n_cams: int = 24, width: int = 320,
         height: int = 240, spp: int = 128) -> Scene:
    """6 x 5 x 3 m room: walls tessellated into 0.1 m squares (25,200
    triangles), 40 boxes (400 triangles), two level-6 icospheres (163,840
    triangles); 3 ceiling lamps and one window; per-vertex cache U[0,2]^3;
    24 cameras at 320 x 240 -> 1,843,200 shading points; 128 spp."""
    return _room_scene("room", seed, 0.1, 6, 1, n_cams, width, height, spp,
                       3, 1, 2002)


def _room_params(target):
    walls_cell = 0.2 if target < 30000 else 0.1
    walls = 2 * 126 / (walls_cell ** 2)
    rem = target - walls
    level = 3
    for L in range(3, 8):
        if 40 * 4 ** L <= 0.5 * rem:
            level = L
    rem -= 40 * 4 ** level
    sub = max(1, int(round(math.sqrt(max(rem, 0) / 400.0))))
    return walls_cell, level, sub


SERVING_TRIANGLES = (20000, 38600, 74600, 144000, 278000, 537000, 1040000, 2000000)


def serving_rooms(seed: int = 1004, n_cams: int = 28, width: int = 320,
                  height: int = 240, counts=SERVING_TRIANGLES, which=None) -> list:
    """Eight rooms with log-spaced triangle counts; each has enough camera
    points (28 x 320 x 240 = 2,150,400) to serve requests of up to 2M
    points as contiguous subsets.  `which` (indices into `counts`) builds
    only those rooms, each identical to its place in the full list."""
    out = []
    for r, target in enumerate(counts):
        if which is not None and r not in which:
            continue
        cell, level, sub = _room_params(target)
        out.append(_room_scene(f"room{r}_{target}", seed * 100 + r, cell, level,
                               sub, n_cams, width, height, 64, 3, 1, 2004))
    return out


def large_room(seed: int = 1005, n_cams: int = 16, width: int = 250,
               height: int = 250, spp: int = 256) -> Scene:
    """About 2M triangles (furniture faces subdivided), 8 emitters (7 lamps
    and a window), 16 cameras at 250 x 250 -> 1,000,000 points, 256 spp."""
    cell, level, sub = _room_params(2000000)
    return _room_scene("large_room", seed, cell, level, sub, n_cams, width,
                       height, spp, 7, 1, 2005)


# --------------------------------------------------------------------------
# material grids, shading tables and observations (differentiation inputs)
# --------------------------------------------------------------------------
def material_grid(res: int = 128, seed: int = 1003) -> np.ndarray:
    """float32 [5, res, res, res] planes a_r, a_g, a_b, roughness, metallic
    (x fastest): albedo U[0,1]^3, roughness U[0.02, 1], metallic U[0,1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.empty((5, res, res, res), dtype=np.float32)
    g[0:3] = rng.uniform(0.0, 1.0, size=(3, res, res, res))
    g[3] = rng.uniform(0.02, 1.0, size=(res, res, res))
    g[4] = rng.uniform(0.0, 1.0, size=(res, res, res))
    return g


def random_shading(n: int, K: int = 6, seed: int = 7) -> np.ndarray:
    """float32 [3 + 6K, n] non-negative shading planes Ld, Ls0[K], Ls1[K]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.empty((3 + 6 * K, n), dtype=np.float32)
    s[0:3] = rng.uniform(0.0, 2.0, size=(3, n))
    s[3:3 + 3 * K] = rng.uniform(0.0, 1.5, size=(3 * K, n))
    s[3 + 3 * K:] = rng.uniform(0.0, 0.3, size=(3 * K, n))
    return s


def random_materials(n: int, seed: int = 8, sigma=SIGMA_GRID) -> np.ndarray:
    """float32 [5, n] per-point a_r, a_g, a_b, roughness, metallic.  A few
    roughness values sit exactly on grid knots and outside the grid so the
    interpolation's clamped and knot cases are exercised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.empty((5, n), dtype=np.float32)
    m[0:3] = rng.uniform(0.0, 1.0, size=(3, n))
    m[3] = rng.uniform(0.0, 1.05, size=n)
    m[4] = rng.uniform(0.0, 1.0, size=n)
    if n >= 32:
        k = rng.choice(n, size=min(n // 8, 4096), replace=False)
        m[3, k] = np.asarray(sigma, np.float32)[rng.integers(0, len(sigma), len(k))]
    return m


def random_observations(n: int, seed: int = 9) -> np.ndarray:
    """float32 [3, n] non-negative observed radiance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 2.0, size=(3, n)).astype(np.float32)


def observation_noise(n: int, seed: int = 10) -> np.ndarray:
    """float32 [3, n] standard normal draws for multiplicative 1% noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(3, n)).astype(np.float32)


def serving_trace(n_requests: int, rate: float, room_points, seed: int = 1104,
                  min_pts: int = 10000, max_pts: int = 2000000,
                  min_spp: int = 16, max_spp: int = 256) -> list:
    """Poisson arrivals at ``rate`` per second.  Each request draws a room
    uniformly, a point count log-uniform in [min_pts, max_pts] taken as a
    contiguous run of that room's camera points, and spp log-uniform in
    [min_spp, max_spp] (rounded).  Returns dicts with arrival time (s),
    room, offset, count, spp and a per-request seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        r = int(rng.integers(0, len(room_points)))
        n = int(round(math.exp(rng.uniform(math.log(min_pts), math.log(max_pts)))))
        n = min(n, int(room_points[r]))
        off = int(rng.integers(0, int(room_points[r]) - n + 1))
        spp = int(round(math.exp(rng.uniform(math.log(min_spp), math.log(max_spp)))))
        out.append(dict(arrival=t, room=r, offset=off, count=n, spp=spp,
                        seed=5000 + i))
    return out


def emitter_schedule(emission: np.ndarray, n_iter: int, seed: int = 2105) -> list:
    """Emitter classification for each of ``n_iter`` iterations of the
    emitter loop: iteration i flags the first (i + 1) / n_iter of the
    emissive triangles in a seeded random order (a stand-in for thresholding
    an emission mask that sharpens over the iterations).  bool [T] each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lit = np.flatnonzero(np.any(emission > 0, axis=0))
    order = rng.permutation(lit)
    out = []
    for i in range(n_iter):
        flags = np.zeros(emission.shape[1], dtype=bool)
        flags[order[: max(1, (len(order) * (i + 1)) // n_iter)]] = True
        out.append(flags)
    return out


def emitter_observations(emission: np.ndarray, tri: np.ndarray, seed: int = 2106) -> np.ndarray:
    """Observed RGB of every pixel for the emission estimate: a pixel whose
    primary hit is an emissive triangle sees its emission with 1 % Gaussian
    multiplicative noise (an emitter reflects nothing); other pixels see
    uniform values in [0, 1].  float32 [3, n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tri = np.asarray(tri)
    n = len(tri)
    obs = rng.uniform(0.0, 1.0, size=(3, n)).astype(np.float32)
    seen = tri >= 0
    lit = np.any(emission > 0, axis=0)
    on = seen.copy()
    on[seen] = lit[tri[seen]]
    obs[:, on] = (emission[:, tri[on]] * (1.0 + 0.01 * rng.standard_normal((3, int(on.sum()))))
                  ).astype(np.float32)
    return obs



def emission_mask(emission: np.ndarray, tri: np.ndarray, seed: int = 2107) -> np.ndarray:
    """Emission mask alpha per pixel for the masked loss, shaped like a mask
    part-way through its optimisation: pixels whose primary hit is an
    emissive triangle get values in [0.5, 1], all others small values in
    [0, 0.02) (most of them below the 0.01 emitter threshold).  float32 [n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tri = np.asarray(tri)
    n = len(tri)
    alpha = (0.02 * rng.random(n) ** 2).astype(np.float32)
    seen = tri >= 0
    lit = np.any(emission > 0, axis=0)
    on = seen.copy()
    on[seen] = lit[tri[seen]]
    alpha[on] = rng.uniform(0.5, 1.0, int(on.sum())).astype(np.float32)
    return alpha


def hashgrid_params(seed: int = 2108) -> np.ndarray:
    """Parameters of the hash-grid material network, laid out as tables
    [32][2^19][2] then W1 [64][64], W2 [64][64], W3 [5][64]: table entries
    U(-1e-4, 1e-4) (the encoding's usual initialisation), weights
    N(0, 1 / 64) (unit gain through each layer).  float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_tab = 32 * (1 << 19) * 2
    n_w = 64 * 64 + 64 * 64 + 5 * 64
    return np.concatenate([rng.uniform(-1e-4, 1e-4, n_tab),
                           rng.standard_normal(n_w) / 8.0]).astype(np.float32)
