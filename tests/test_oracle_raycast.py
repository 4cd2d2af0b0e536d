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
