"""The bake's random streams and its ray cast, each checked on its own
through the C ABI against the oracle: the stratified lobe uniforms bit for
bit over 2^20 counters per case (key and point index above 32 bits), and
the closest hit of 2^16 random rays against brute force over every
triangle."""
import numpy as np
import pytest
import torch

import synth
from oracle import bake as ob
from paper_2304_05669_amd import fipt

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("lobe,n_s", [(0, 1024), (3, 100), (16, 1)])
def test_lobe_uniforms_bitwise(lobe, n_s):
    seed = 0x0123456789ABCDEF
    p0 = (1 << 32) - 500                     # the point index crosses into the high word
    n_pts = (1 << 20) // n_s
    got = fipt.fipt_lobe_uniforms(seed, p0, n_pts, lobe, n_s).cpu().numpy()
    p = p0 + np.repeat(np.arange(n_pts, dtype=np.int64), n_s)
    s = np.tile(np.arange(n_s, dtype=np.int64), n_pts)
    want1, want2 = ob.lobe_uniforms(seed, p, lobe, s, n_s)
    np.testing.assert_array_equal(got[0].reshape(-1), want1.astype(np.float32))
    np.testing.assert_array_equal(got[1].reshape(-1), want2.astype(np.float32))


def _mesh():
    """Closed unit box (the tiny box's 20 triangles) around an icosphere of
    5120 triangles: a BVH several levels deep, inside and outside faces."""
    box = synth.tiny_box()
    sv, st = synth.icosphere(4)
    sv = (0.5 + 0.3 * sv).astype(np.float32)
    verts = np.concatenate([box.verts, sv]).astype(np.float32)
    tris = np.concatenate([box.tris, st + len(box.verts)]).astype(np.int32)
    return verts, tris


# (scale, offset): the mesh and ray origins are mapped by x -> scale x + offset,
# so the node bounds' single exponent and origins are exercised far from the
# unit cube (large coordinates with small extents, and a sub-millimetre scene)
TRANSFORMS = {
    "unit": (1.0, (0.0, 0.0, 0.0)),
    "far": (1000.0, (2.0e4, -3.0e4, 1.0e4)),
    "small": (1.0e-4, (1.0e-4, 3.0e-4, -2.0e-4)),
}


@pytest.mark.parametrize("frame", list(TRANSFORMS))
def test_cast_rays_match_brute_force(frame):
    scale, offset = TRANSFORMS[frame]
    verts, tris = _mesh()
    verts = (verts.astype(np.float64) * scale + np.array(offset)).astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(77))
    n = 1 << 16
    o = rng.uniform(0.02, 0.98, size=(n, 3))
    d = rng.standard_normal(size=(n, 3))
    k = n // 64
    d[np.arange(k), rng.integers(0, 3, size=k)] = 0.0             # axis-parallel components
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # a few rays from outside the box, pointing away from it: misses
    o[-256:] = rng.uniform(1.5, 2.0, size=(256, 3))
    d[-256:] = np.abs(d[-256:]) + 0.1
    o = o * scale + np.array(offset)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    scene = fipt.Scene(verts, tris, device=0)
    try:
        rays = torch.from_numpy(np.concatenate([o32.T, d32.T]).copy()).to(DEV)
        tri, tuv = fipt.fipt_cast_rays(scene, rays)
        torch.cuda.synchronize()
        tri = tri.cpu().numpy()
        tuv = tuv.cpu().numpy()
    finally:
        scene.destroy()
    sc = synth.Scene(name="rays", verts=verts, tris=tris, cache_kind="triangle",
                     cache=np.zeros((3, len(tris)), np.float32),
                     emission=np.zeros((3, len(tris)), np.float32))
    # the oracle's ambiguity band tol_rel (1 + t) is sized for unit scenes:
    # scale it with a smaller scene so it covers the same relative width
    osc = ob.OracleScene(sc, tol_rel=1e-5 * min(scale, 1.0))
    w_tri, w_t, w_b, n_cand = ob.cast(osc, o32.astype(np.float64), d32.astype(np.float64))
    assert (tri[-256:] == -1).all() and (w_tri[-256:] == -1).all()
    clear = n_cand <= 1
    assert clear.mean() > 0.995
    np.testing.assert_array_equal(tri[clear], w_tri[clear])
    hit = clear & (w_tri >= 0)
    np.testing.assert_allclose(tuv[0, hit], w_t[hit], rtol=2e-5, atol=1e-6 * scale)
    np.testing.assert_allclose(tuv[1, hit], w_b[hit, 0], atol=2e-4)
    np.testing.assert_allclose(tuv[2, hit], w_b[hit, 1], atol=2e-4)
    # inside the tie band the GPU still reports a hit of similar distance
    amb = ~clear
    assert (tri[amb] >= 0).all()
    np.testing.assert_allclose(tuv[0, amb], w_t[amb], rtol=1e-3, atol=1e-5 * scale)
