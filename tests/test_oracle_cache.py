"""Pins of the oracle's voxel radiance cache (Sec. 4.2, the query of Eq. 9):

* voxel indices by hand: interior points, points on a face (the upper
  voxel), on the box's far face and outside the box (the border voxels);
* pooling against a pure-Python brute force (dictionary of lists, mean per
  voxel) on small random inputs, counts summing to the number of points,
  constant observations giving that constant in every occupied voxel;
* the C oracle's nearest-voxel query: rays from inside the unit box to
  points of its walls computed in closed form return the value of the
  voxel the hit point falls in plus the wall's emission, for a cache whose
  voxel values encode their own (i, j, k);
* furnace: a constant voxel cache in the closed box gives Ld = L exactly,
  as the per-triangle cache does;
* a hit on a voxel face is flagged and its envelope spans both voxels.
"""
import copy
import math

import numpy as np
import pytest

import synth
from oracle import bake as ob
from oracle import cache as oc


def test_voxel_index_by_hand():
    lo, hi, R = (0.0, 0.0, 0.0), (1.0, 2.0, 4.0), 4
    pts = np.array([
        [0.1, 0.3, 0.6],      # (0, 0, 0)
        [0.3, 0.6, 2.5],      # (1, 1, 2)
        [0.25, 0.5, 1.0],     # on faces: (1, 1, 1)
        [1.0, 2.0, 4.0],      # far corner: (3, 3, 3)
        [-5.0, 9.0, 1.5],     # outside: (0, 3, 1)
        [0.99, 0.01, 3.99],   # (3, 0, 3)
    ]).T
    want = [(0, 0, 0), (1, 1, 2), (1, 1, 1), (3, 3, 3), (0, 3, 1), (3, 0, 3)]
    got = oc.voxel_of(pts, lo, hi, R)
    assert list(got) == [(k * R + j) * R + i for i, j, k in want]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pool_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n, R = 500, 5
    lo, hi = np.array([-1.0, 0.0, 2.0]), np.array([1.0, 0.5, 3.0])
    x = lo[:, None] + rng.uniform(-0.1, 1.1, size=(3, n)) * (hi - lo)[:, None]
    obs = rng.uniform(0, 4, size=(3, n))
    cache, counts = oc.voxel_pool(x, obs, lo, hi, R)
    assert counts.sum() == n
    groups = {}
    for p in range(n):
        ijk = []
        for a in range(3):
            u = (x[a, p] - lo[a]) / (hi[a] - lo[a]) * R
            ijk.append(min(max(int(math.floor(u)), 0), R - 1))
        groups.setdefault((ijk[2] * R + ijk[1]) * R + ijk[0], []).append(p)
    want = np.zeros((3, R ** 3))
    for v, ps in groups.items():
        assert counts[v] == len(ps)
        for c in range(3):
            want[c, v] = sum(obs[c, p] for p in ps) / len(ps)
    empty = np.setdiff1d(np.arange(R ** 3), list(groups))
    assert np.all(counts[empty] == 0) and np.all(cache[:, empty] == 0.0)
    np.testing.assert_allclose(cache, want, rtol=1e-14, atol=0)


def test_pool_of_a_constant_is_that_constant():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(3, 2000))
    obs = np.full((3, 2000), 0.1)
    cache, counts = oc.voxel_pool(x, obs, (0, 0, 0), (1, 1, 1), 6)
    np.testing.assert_allclose(cache[:, counts > 0], 0.1, rtol=1e-14)


def _coded_cache(R):
    """Voxel (i, j, k) holds (i, 100 + j, 1000 + k): a query tells which
    voxel it read."""
    i, j, k = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    cache = np.zeros((3, R, R, R), np.float32)        # [c][k][j][i]
    cache[0] = np.transpose(i, (2, 1, 0))
    cache[1] = 100 + np.transpose(j, (2, 1, 0))
    cache[2] = 1000 + np.transpose(k, (2, 1, 0))
    return cache.reshape(3, -1)


def test_nearest_voxel_query_on_the_walls():
    sc = copy.deepcopy(synth.tiny_box())
    sc.emission[:] = 0
    R = 8
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(_coded_cache(R), R, (0, 0, 0), (1, 1, 1))
    rng = np.random.default_rng(4)
    o = np.array([0.5, 0.45, 0.4])
    n = 400
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # exit point of the unit cube in closed form
    with np.errstate(divide="ignore"):
        t_exit = np.min(np.where(d > 0, (1 - o) / d, np.where(d < 0, -o / d, np.inf)), axis=1)
    x = o + t_exit[:, None] * d
    ijk = np.clip(np.floor(x * R), 0, R - 1)
    frac = x * R - np.floor(x * R)
    interior = np.all((frac > 1e-6) & (frac < 1 - 1e-6) | (np.abs(x - np.round(x)) < 1e-12), axis=1)
    got = ob.trace_radiance(osc, np.tile(o, (n, 1)), d)
    want = np.stack([ijk[:, 0], 100 + ijk[:, 1], 1000 + ijk[:, 2]], axis=1)
    assert interior.sum() > 350
    np.testing.assert_array_equal(got[interior], want[interior])


def test_voxel_query_adds_emission():
    sc = copy.deepcopy(synth.tiny_box())
    R = 4
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(np.full((3, R ** 3), 0.25, np.float32), R, (0, 0, 0), (1, 1, 1))
    # straight up through the emitter quad [0.375, 0.625]^2 at z = 1
    got = ob.trace_radiance(osc, np.array([[0.5, 0.5, 0.5]]), np.array([[0.0, 0.0, 1.0]]))
    np.testing.assert_array_equal(got[0], [10.25, 10.25, 10.25])


def test_constant_voxel_furnace(tiny, tiny_points):
    pts, tri, _ = tiny_points
    sc = copy.deepcopy(tiny)
    sc.emission[:] = 0
    L = np.float32(0.7)
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(np.full((3, 16 ** 3), L, np.float32), 16, (0, 0, 0), (1, 1, 1))
    r = ob.bake(osc, pts, tri, spp_d=64, spp_s=8, seed=sc.seed)
    valid = tri >= 0
    clean = np.all(r["hi"] - r["lo"] == 0.0, axis=0) & valid
    assert clean.sum() > 4000
    np.testing.assert_allclose(r["mean"][0:3, clean], float(L), rtol=1e-14)
    amb = valid & ~clean
    assert np.all(r["lo"][0:3, amb] <= L + 1e-12) and np.all(r["hi"][0:3, amb] >= L - 1e-12)


def test_face_hits_span_both_voxels():
    """Rays that end on the face x = 0.5 between two voxels of a 2^3 grid:
    the nominal value is the upper voxel's, and a bake whose samples land
    there reports the other voxel inside its envelope."""
    sc = copy.deepcopy(synth.tiny_box())
    sc.emission[:] = 0
    R = 2
    osc = ob.OracleScene(sc)
    osc.set_voxel_cache(_coded_cache(R), R, (0, 0, 0), (1, 1, 1))
    # a ray to the floor point (0.5, 0.25, 0): exactly on the face i = 0 | 1
    got = ob.trace_radiance(osc, np.array([[0.5, 0.25, 0.5]]), np.array([[0.0, 0.0, -1.0]]))
    np.testing.assert_array_equal(got[0], [1, 100, 1000])
    # a floor point whose mirror direction (roughness 1e-3) ends on the
    # ceiling at x = 0.5, the face between voxels i = 0 and i = 1
    pts = np.zeros((9, 1), np.float32)
    pts[0:3, 0] = (0.3 + 0.2e-4, 0.25, 0.0)        # + 0.2 eps: the ray starts eps above
    pts[5, 0] = 1.0
    wo = np.array([-0.2, 0.0, 1.0]) / math.hypot(0.2, 1.0)
    pts[6:9, 0] = wo
    r = ob.bake(osc, pts, np.array([0], np.int32), spp_d=16, spp_s=64, sigma=[1e-3], seed=5)
    assert r["n_ambiguous"] >= 60
    ls0 = slice(3, 6)
    # channel 0 encodes i: the envelope holds both voxels' values
    assert r["hi"][3, 0] - r["lo"][3, 0] > 0.5 * r["hi"][3, 0] > 0
    assert np.all(r["lo"][ls0] <= r["mean"][ls0]) and np.all(r["mean"][ls0] <= r["hi"][ls0])
