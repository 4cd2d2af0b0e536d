"""Pins of the oracle's brute-force ray caster: analytic hits inside a closed
axis-aligned box, and hand cases (behind the origin, parallel, vertex and
edge hits, near misses)."""
import numpy as np

import synth
from oracle import bake as ob


def _single_triangle():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    t = np.array([[0, 1, 2]], np.int32)
    return synth.Scene(name="one", verts=v, tris=t, cache_kind="triangle",
                       cache=np.ones((3, 1), np.float32),
                       emission=np.zeros((3, 1), np.float32))


def test_box_hits_match_slab_distance(tiny, tiny_oracle):
    rng = np.random.default_rng(21)
    n = 4000
    o = rng.uniform(0.05, 0.95, size=(n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # exact distance to the unit cube's walls from inside
    with np.errstate(divide="ignore"):
        tw = np.where(d > 0, (1.0 - o) / d, np.where(d < 0, -o / d, np.inf))
    t_exact = tw.min(axis=1)
    axis = tw.argmin(axis=1)
    tri, t, b, nc = ob.cast(tiny_oracle, o, d)
    assert (tri >= 0).all()
    np.testing.assert_allclose(t, t_exact, rtol=1e-12, atol=1e-13)
    hit = o + t[:, None] * d
    V = tiny.verts.astype(np.float64)
    for q in range(n):
        tv = V[tiny.tris[tri[q]]]
        a = axis[q]
        side = 1.0 if d[q, a] > 0 else 0.0
        # the triangle lies in the wall that the slab test picked
        assert np.all(tv[:, a] == side)
        lo, hi = tv.min(0), tv.max(0)
        assert np.all(hit[q] >= lo - 1e-12) and np.all(hit[q] <= hi + 1e-12)


def test_hand_cases():
    sc = _single_triangle()
    osc = ob.OracleScene(sc)
    down = np.array([0.0, 0.0, -1.0])
    cases = [
        # origin, direction, expected triangle, minimum outcome count
        ((0.25, 0.25, 1.0), down, 0, 1),               # clean interior hit
        ((0.25, 0.25, -1.0), down, -1, 1),             # triangle behind the origin
        ((0.25, 0.25, 1.0), (1.0, 0.0, 0.0), -1, 1),   # parallel to the plane
        ((0.0, 0.0, 1.0), down, 0, 2),                 # through a vertex: hit or miss
        ((0.5, 0.5, 1.0), down, 0, 2),                 # on the hypotenuse
        ((0.5 + 1e-3, 0.5 + 1e-3, 1.0), down, -1, 1),  # clear miss past the edge
        ((0.25, -1e-3, 1.0), down, -1, 1),             # clear miss below the edge
    ]
    for o, d, exp_tri, min_nc in cases:
        tri, t, b, nc = ob.cast(osc, np.array(o, float), np.array(d, float))
        assert tri[0] == exp_tri, (o, d)
        assert nc[0] >= min_nc, (o, d)
        if exp_tri == 0:
            assert abs(t[0] - o[2]) < 1e-15
    # a ray through the shared diagonal of two coplanar triangles is a hit
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    t2 = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    sq = synth.Scene(name="quad", verts=v, tris=t2, cache_kind="triangle",
                     cache=np.ones((3, 2), np.float32), emission=np.zeros((3, 2), np.float32))
    osq = ob.OracleScene(sq)
    xs = np.linspace(0.01, 0.99, 97)
    o = np.stack([xs, xs, np.ones_like(xs)], 1)
    d = np.tile(down, (len(xs), 1))
    tri, t, b, nc = ob.cast(osq, o, d)
    assert (tri >= 0).all() and (nc >= 2).all()


def test_nearest_of_stacked_planes():
    """Three parallel squares at z = 0, 1, 2: a downward ray from above hits
    the top one, an upward ray from below the bottom one, with ties to the
    lower index for coincident copies."""
    quads = []
    for z in (0.0, 1.0, 2.0, 2.0):
        quads.append([[-1, -1, z], [1, -1, z], [1, 1, z], [-1, 1, z]])
    v = np.array(quads, np.float32).reshape(-1, 3)
    tris = []
    for q in range(4):
        tris += [[4 * q, 4 * q + 1, 4 * q + 2], [4 * q, 4 * q + 2, 4 * q + 3]]
    tris = np.array(tris, np.int32)
    sc = synth.Scene(name="stack", verts=v, tris=tris, cache_kind="triangle",
                     cache=np.ones((3, 8), np.float32), emission=np.zeros((3, 8), np.float32))
    osc = ob.OracleScene(sc)
    tri, t, _, _ = ob.cast(osc, np.array([0.3, -0.2, 5.0]), np.array([0.0, 0.0, -1.0]))
    assert tri[0] in (4, 5) and abs(t[0] - 3.0) < 1e-15
    tri, t, _, _ = ob.cast(osc, np.array([0.3, -0.2, -5.0]), np.array([0.0, 0.0, 1.0]))
    assert tri[0] in (0, 1) and abs(t[0] - 5.0) < 1e-15


def test_radiance_lookup():
    """Per-vertex cache linear in position -> the interpolated radiance at a
    hit equals that linear function at the hit point; per-triangle cache
    plus emission is their sum; a miss is zero."""
    rng = np.random.default_rng(8)
    sc = synth.room(n_cams=1, width=4, height=4)
    A = rng.uniform(0.1, 0.5, size=(3, 3))
    b = rng.uniform(0.0, 1.0, size=3)
    V = sc.verts.astype(np.float64)
    sc.cache = (A @ V.T + b[:, None]).astype(np.float32)
    sc.emission[:] = 0
    osc = ob.OracleScene(sc)
    o = np.tile(np.array([3.0, 2.5, 1.5]), (500, 1)) + rng.uniform(-0.2, 0.2, (500, 3))
    d = rng.standard_normal((500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tri, t, _, _ = ob.cast(osc, o, d)
    R = ob.trace_radiance(osc, o, d)
    x = o + t[:, None] * d
    # cache values are float32-rounded; compare at that precision
    want = x @ A.T + b
    np.testing.assert_allclose(R, want, rtol=2e-6, atol=2e-6)

    tiny = synth.tiny_box()
    ot = ob.OracleScene(tiny)
    up = np.array([[0.5, 0.5, 0.5]]), np.array([[0.0, 0.0, 1.0]])   # hits the emitter
    tri, _, _, _ = ob.cast(ot, *up)
    R = ob.trace_radiance(ot, *up)[0]
    np.testing.assert_array_equal(R, tiny.cache[:, tri[0]].astype(np.float64) + 10.0)
    side = np.array([[0.5, 0.5, 0.5]]), np.array([[1.0, 0.0, 0.0]])
    tri, _, _, _ = ob.cast(ot, *side)
    np.testing.assert_array_equal(ob.trace_radiance(ot, *side)[0], tiny.cache[:, tri[0]])
    one = _single_triangle()
    oo = ob.OracleScene(one)
    np.testing.assert_array_equal(ob.trace_radiance(oo, np.array([0.2, 0.2, 1.0]), np.array([0.0, 0.0, 1.0])), 0.0)


def test_closed_mesh_is_watertight_at_shared_edges():
    """A ray that meets a shared edge of a closed surface hits it: in exact
    arithmetic the closed barycentric test accepts the edge on both
    triangles.  Float64 rounding can reject it on both (about one ray in
    eight aimed exactly at an edge); the oracle then reports the nearest
    triangle within its tolerance band, with barycentrics clamped onto it.
    Rays from inside a closed icosphere aimed at points of every shared edge
    must all hit, at the distance to that point, on one of the two triangles
    of the edge, and report the other outcome as possible."""
    v, f = synth.icosphere(2)
    verts = (v * 1.5 + 0.25).astype(np.float32)
    tris = f.astype(np.int32)
    sc = synth.Scene(name="ico", verts=verts, tris=tris, cache_kind="triangle",
                     cache=np.ones((3, len(tris)), np.float32),
                     emission=np.zeros((3, len(tris)), np.float32))
    osc = ob.OracleScene(sc)
    # every edge and the two triangles that share it
    owners = {}
    for t_i, tri in enumerate(tris):
        for a, b in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])):
            owners.setdefault((min(a, b), max(a, b)), []).append(t_i)
    edges = sorted(owners)
    assert all(len(owners[e]) == 2 for e in edges)
    rng = np.random.default_rng(77)
    V = verts.astype(np.float64)
    o_all, d_all, want_t, pairs = [], [], [], []
    for (a, b) in edges:
        for s in rng.uniform(0.02, 0.98, size=8):
            tgt = V[a] + s * (V[b] - V[a])
            o = V.mean(0) + rng.uniform(-0.3, 0.3, size=3)
            d = tgt - o
            o_all.append(o)
            d_all.append(d / np.linalg.norm(d))
            want_t.append(np.linalg.norm(d))
            pairs.append(owners[(a, b)])
    tri, t, bary, nc = ob.cast(osc, np.array(o_all), np.array(d_all))
    pairs = np.array(pairs)
    assert (tri >= 0).all(), f"{int((tri < 0).sum())} of {len(tri)} edge rays missed"
    assert ((tri == pairs[:, 0]) | (tri == pairs[:, 1])).all()
    np.testing.assert_allclose(t, want_t, rtol=1e-9)
    assert (bary >= 0).all() and (bary.sum(1) <= 1 + 1e-15).all()
    assert (nc >= 2).all()


def test_silhouette_near_miss_outcomes():
    """Past the free edge of a lone triangle: inside the tolerance band the
    nominal result is a hit clamped onto the edge with a miss among the
    possible outcomes; beyond the band it is a plain miss with one outcome."""
    osc = ob.OracleScene(_single_triangle())
    down = np.array([[0.0, 0.0, -1.0]])
    for off in (1e-9, 1e-7):
        tri, t, bary, nc = ob.cast(osc, np.array([[0.5 + off, 0.5 + off, 1.0]]), down)
        assert tri[0] == 0 and nc[0] >= 2 and abs(t[0] - 1.0) < 1e-15
        assert abs(bary[0].sum() - 1.0) < 1e-15 and (bary[0] >= 0).all()
    tri, t, bary, nc = ob.cast(osc, np.array([[0.5 + 1e-4, 0.5 + 1e-4, 1.0]]), down)
    assert tri[0] == -1 and nc[0] == 1


def test_candidate_overflow_is_an_error():
    """More coincident surfaces along one ray than the oracle keeps outcomes
    for (256): the cast is refused, not truncated."""
    import pytest
    n = 300
    v = np.tile(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), (n, 1))
    t = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    sc = synth.Scene(name="pile", verts=v, tris=t, cache_kind="triangle",
                     cache=np.ones((3, n), np.float32), emission=np.zeros((3, n), np.float32))
    osc = ob.OracleScene(sc)
    with pytest.raises(ob.CandidateOverflow):
        ob.cast(osc, np.array([0.25, 0.25, 1.0]), np.array([0.0, 0.0, -1.0]))
    with pytest.raises(ob.CandidateOverflow):
        ob.trace_radiance(osc, np.array([0.25, 0.25, 1.0]), np.array([0.0, 0.0, -1.0]))
    pts = np.zeros((9, 1), np.float32)
    pts[0:3, 0] = (0.25, 0.25, 0.5)
    pts[3:6, 0] = (0.0, 0.0, -1.0)
    pts[6:9, 0] = (0.0, 0.0, -1.0)
    with pytest.raises(ob.CandidateOverflow):
        ob.bake(osc, pts, np.zeros(1, np.int32), spp_d=64, spp_s=1, sigma=(0.5,), seed=1)
    # below the limit: fine, with every copy among the outcomes
    few = synth.Scene(name="pile", verts=v[:60], tris=t[:20], cache_kind="triangle",
                      cache=np.ones((3, 20), np.float32), emission=np.zeros((3, 20), np.float32))
    tri, tt, _, nc = ob.cast(ob.OracleScene(few), np.array([0.25, 0.25, 1.0]), np.array([0.0, 0.0, -1.0]))
    assert tri[0] == 0 and nc[0] == 20
