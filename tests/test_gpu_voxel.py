"""GPU parity of the voxel radiance cache (Sec. 4.2): pooling of observed
pixels onto the grid against the oracle (bit for bit), and the bake's
nearest-voxel query against the oracle's bake, through the C ABI.

Sizes: pooling from 1 to 1,843,200 pixels (the room's shading points) on
grids of 1^3 to 256^3; the bake on the whole tiny box (4096 points, 448
lobe samples each) and on sampled points of the full room with a 256^3
grid, the configuration the benchmark times."""
import copy

import numpy as np
import pytest
import torch

import synth
from oracle import bake as ob
from oracle import cache as oc
from paper_2304_05669_amd import fipt
from tests.parity import assert_bake_parity, bake_report, oracle_bake_chunked, stratified_points

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _smooth_cache(R):
    """A cache linear in the voxel index, distinct per channel: neighbouring
    voxels differ by at most 0.0015, so a hit that single precision places
    in the neighbour of the oracle's voxel moves a point's mean by ~1e-6,
    while a transposed or shifted index is off by up to ~0.4."""
    g = 0.064 / R
    k, j, i = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    c = np.stack([1.0 + g * (i + 2 * j + 3 * k), 0.5 + g * (3 * i + j + 2 * k),
                  2.0 + g * (2 * i + 3 * j + k)])
    return c.reshape(3, -1).astype(np.float32)


@pytest.mark.parametrize("n,R", [(1, 1), (1000, 7), (100003, 64), (250000, 256), (50000, 512)])
def test_voxel_pool_bitwise(n, R):
    rng = np.random.default_rng(n + R)
    lo = np.array([-1.0, 0.5, 2.0], np.float32)
    hi = np.array([2.0, 1.5, 2.25], np.float32)
    # clustered on a few planes like surface points, some outside the box
    x = lo[:, None] + rng.uniform(-0.05, 1.05, size=(3, n)) * (hi - lo)[:, None]
    x[2, : n // 3] = lo[2]
    x[0, n // 3: n // 2] = hi[0]
    x = x.astype(np.float32)
    obs = rng.uniform(0, 5, size=(3, n)).astype(np.float32)
    plan = fipt.VoxelPlan(x, R, lo, hi)
    out = torch.full((3, R ** 3), float("nan"), dtype=torch.float32, device=DEV)
    got = plan.pool(_t(obs), out=out)
    again = plan.pool(_t(obs))
    torch.cuda.synchronize()
    want, counts = oc.voxel_pool(x, obs, lo, hi, R)
    g = got.cpu().numpy()
    assert np.array_equal(g, want.astype(np.float32))
    assert torch.equal(got, again)
    assert counts.sum() == n


def test_voxel_pool_room_pixels():
    """The room's 1,843,200 shading points pooled onto 256^3 voxels."""
    sc = synth.room()
    scene = fipt.Scene(sc.verts, sc.tris, device=0)
    planes, tri = fipt.fipt_gen_points(scene, sc.cameras)
    torch.cuda.synchronize()
    pos = planes[0:3].cpu().numpy()
    obs = synth.random_observations(sc.n_points, seed=51)
    plan = fipt.VoxelPlan(pos, 256, sc.bmin, sc.bmax)
    got = plan.pool(_t(obs))
    torch.cuda.synchronize()
    want, counts = oc.voxel_pool(pos, obs, sc.bmin, sc.bmax, 256)
    assert np.array_equal(got.cpu().numpy(), want.astype(np.float32))
    assert (counts > 0).sum() > 100000
    scene.destroy()


def _voxel_scene(sc, cache, R, lo, hi, emission=True):
    s = fipt.Scene(sc.verts, sc.tris, device=0)
    s.set_voxel_radiance(_t(cache), R, lo, hi,
                         _t(sc.emission) if emission else None)
    return s


@pytest.mark.parametrize("R", [32, 30, 1])
def test_voxel_bake_parity_tiny(tiny, tiny_points, R):
    """R = 30 leaves the last brick of each axis partly outside the grid;
    R = 1 is a single voxel."""
    pts, tri, _ = tiny_points
    cache = _smooth_cache(R)
    s = _voxel_scene(tiny, cache, R, tiny.bmin, tiny.bmax)
    assert s.info().cache_kind == fipt.CACHE_VOXEL
    got = fipt.fipt_bake(s, _t(pts), _t(tri, torch.int32), tiny.spp, tiny.spp, tiny.sigma,
                         tiny.seed)
    torch.cuda.synchronize()
    osc = ob.OracleScene(tiny)
    osc.set_voxel_cache(cache, R, tiny.bmin, tiny.bmax)
    want = ob.bake(osc, pts, tri, spp_d=tiny.spp, spp_s=tiny.spp, seed=tiny.seed)
    r = assert_bake_parity(got.cpu().numpy(), want)
    print(f"tiny box voxel parity (R = {R}):", r)
    s.destroy()


def test_voxel_bake_parity_room_sampled():
    """Full-size room bake with a 256^3 voxel cache (the benchmark's launch);
    oracle on sampled points baking identical inputs."""
    sc = synth.room()
    R = 256
    cache = _smooth_cache(R)
    s = _voxel_scene(sc, cache, R, sc.bmin, sc.bmax)
    planes, tri_g = fipt.fipt_gen_points(s, sc.cameras)
    torch.cuda.synchronize()
    idx = stratified_points(sc.n_points, 1024, 47)
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(cache, R, sc.bmin, sc.bmax)
    prim = ob.primary(osc, idx=idx)
    p32, t32 = ob.points_f32(prim)
    ii = torch.from_numpy(idx).to(DEV)
    planes[:, ii] = _t(p32)
    tri_g[ii] = _t(t32, torch.int32)
    out = fipt.fipt_bake(s, planes, tri_g, sc.spp, sc.spp, sc.sigma, sc.seed)
    torch.cuda.synchronize()
    got = out[:, ii].cpu().numpy()
    full_p = np.zeros((9, sc.n_points), np.float32)
    full_t = np.full(sc.n_points, -1, np.int32)
    full_p[:, idx] = p32
    full_t[idx] = t32
    want = oracle_bake_chunked(ob.bake, osc, full_p, full_t, idx, label="voxel room",
                               spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed)
    print("room voxel parity:", bake_report(got, want))
    assert_bake_parity(got, want)
    s.destroy()


def test_pooled_cache_end_to_end_tiny(tiny, tiny_points):
    """Observations of the tiny box (its per-triangle cache plus emission at
    every pixel) pooled onto 16^3 voxels and baked: the pooled grid equals
    the oracle's bit for bit, and the bake matches the oracle's bake with
    that grid.  A pooled grid is not smooth, so a hit that single precision
    puts in the neighbouring voxel can move a point by more than 1e-4: at
    least 99 % of points must be within 1e-4, the rest inside the envelope."""
    pts, tri, _ = tiny_points
    R = 16
    seen = tri >= 0
    obs = np.zeros((3, len(tri)), np.float32)
    obs[:, seen] = tiny.cache[:, tri[seen]] + tiny.emission[:, tri[seen]]
    plan = fipt.VoxelPlan(pts[0:3], R, tiny.bmin, tiny.bmax)
    cache = plan.pool(_t(obs))
    torch.cuda.synchronize()
    want_c, _ = oc.voxel_pool(pts[0:3], obs, tiny.bmin, tiny.bmax, R)
    assert np.array_equal(cache.cpu().numpy(), want_c.astype(np.float32))
    # L' already holds what the emitter's pixels saw: no separate emission
    s = fipt.Scene(tiny.verts, tiny.tris, device=0)
    s.set_voxel_radiance(cache, R, tiny.bmin, tiny.bmax)
    got = fipt.fipt_bake(s, _t(pts), _t(tri, torch.int32), 64, 64, tiny.sigma, 3)
    torch.cuda.synchronize()
    sc = copy.deepcopy(tiny)
    sc.emission[:] = 0
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(want_c.astype(np.float32), R, tiny.bmin, tiny.bmax)
    want = ob.bake(osc, pts, tri, spp_d=64, spp_s=64, seed=3)
    r = assert_bake_parity(got.cpu().numpy(), want, min_frac=0.99)
    print("tiny box pooled voxel parity:", r)
    s.destroy()


def test_switching_caches(tiny, tiny_points):
    """A scene returns to its per-triangle cache bit for bit after a voxel
    cache, and a second, larger voxel grid replaces the first."""
    pts, tri, _ = tiny_points
    s = fipt.Scene(tiny.verts, tiny.tris, device=0)
    cache, em = _t(tiny.cache), _t(tiny.emission)
    s.set_radiance(cache, fipt.CACHE_TRIANGLE, em)
    P, T = _t(pts), _t(tri, torch.int32)
    a = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 9).clone()
    s.set_voxel_radiance(_t(_smooth_cache(4)), 4, tiny.bmin, tiny.bmax, em)
    b = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 9).clone()
    s.set_voxel_radiance(_t(_smooth_cache(8)), 8, tiny.bmin, tiny.bmax, em)
    c = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 9).clone()
    s.set_radiance(cache, fipt.CACHE_TRIANGLE, em)
    d = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 9).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, d)
    assert not torch.equal(a, b) and not torch.equal(b, c)
    assert s.info().cache_kind == fipt.CACHE_TRIANGLE
    s.destroy()


def test_voxel_arguments_rejected(tiny, tiny_points):
    pts, tri, _ = tiny_points
    s = fipt.Scene(tiny.verts, tiny.tris, device=0)
    c = _t(_smooth_cache(4))
    # res = 0: the binding's shape check or the library's range check
    with pytest.raises((ValueError, fipt.FiptError)):
        s.set_voxel_radiance(_t(np.zeros((3, 1), np.float32)), 0, tiny.bmin, tiny.bmax)
    with pytest.raises(fipt.FiptError):
        s.set_voxel_radiance(c, 4, tiny.bmax, tiny.bmin)
    with pytest.raises(ValueError):
        s.set_voxel_radiance(c, 5, tiny.bmin, tiny.bmax)
    with pytest.raises(fipt.FiptError):
        fipt.VoxelPlan(pts[0:3], 513, tiny.bmin, tiny.bmax)
    plan = fipt.VoxelPlan(pts[0:3], 4, tiny.bmin, tiny.bmax)
    with pytest.raises(ValueError):
        plan.pool(torch.zeros((3, pts.shape[1] - 1), device=DEV))
    with pytest.raises(ValueError):
        plan.pool(torch.zeros((3, pts.shape[1]), device=DEV), out=torch.zeros((3, 63), device=DEV))
    srv = fipt.Server(device=0, pool_bytes=64 << 20, max_inflight=4, samples_per_launch=1 << 20)
    # a scene that serving requests reference cannot change to a voxel cache
    s.set_radiance(_t(tiny.cache), fipt.CACHE_TRIANGLE, _t(tiny.emission))
    P, T = _t(pts), _t(tri, torch.int32)
    t = srv.submit(s, P, T, 8, 8, tiny.sigma, 1)
    assert srv.wait(t, timeout_s=60.0)
    with pytest.raises(fipt.FiptError):
        s.set_voxel_radiance(c, 4, tiny.bmin, tiny.bmax)
    with pytest.raises(fipt.FiptError):
        s.set_radiance(_t(tiny.cache), fipt.CACHE_TRIANGLE, _t(tiny.emission))
    with pytest.raises(fipt.FiptError):
        s.set_emission(_t(tiny.emission))
    srv.release(t)
    # serving bakes per-triangle and per-vertex caches only
    s.set_voxel_radiance(c, 4, tiny.bmin, tiny.bmax)
    with pytest.raises(fipt.FiptError):
        srv.submit(s, P, T, 8, 8, tiny.sigma, 1)
    srv.destroy()
    s.destroy()


def test_empty_voxel_grid_reads_emission_only(tiny, tiny_points):
    """An all-zero grid has no occupied voxel: every hit reads the emission
    alone, bit for bit what a per-triangle cache of zeros gives."""
    pts, tri, _ = tiny_points
    s = fipt.Scene(tiny.verts, tiny.tris, device=0)
    em = _t(tiny.emission)
    P, T = _t(pts), _t(tri, torch.int32)
    s.set_radiance(torch.zeros((3, tiny.n_tris), dtype=torch.float32, device=DEV),
                   fipt.CACHE_TRIANGLE, em)
    a = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 4).clone()
    s.set_voxel_radiance(torch.zeros((3, 8 ** 3), dtype=torch.float32, device=DEV), 8, tiny.bmin,
                         tiny.bmax, em)
    b = fipt.fipt_bake(s, P, T, 32, 32, tiny.sigma, 4).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert float(a.abs().max()) > 0
    s.destroy()
