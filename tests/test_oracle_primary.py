"""Pins of the oracle's shading points (camera rays through pixel centres,
closest hit, face normal toward the viewer, wo = -dir) by geometric
properties of a pinhole camera facing a flat wall:

* hit points on the wall form a regular grid with equal horizontal and
  vertical pitch (square pixels, any aspect ratio);
* the two central pixel columns straddle the view axis symmetrically;
* image rows run downward (row 0 is the top);
* the angle between the top and bottom pixel-centre rays of a column is
  2 atan(tan(vfov/2) (1 - 1/H));
* the normal faces the camera and wo points back at it.
"""
import math

import numpy as np

import synth
from oracle import bake as ob


def _wall_scene(W, H, vfov=50.0):
    # a large wall at y = 4 seen from the origin looking +y
    v = np.array([[-50, 4, -50], [50, 4, -50], [50, 4, 50], [-50, 4, 50]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    cam = synth.Camera(pos=(0.0, 0.0, 0.0), fwd=(0.0, 1.0, 0.0), up=(0.0, 0.0, 1.0),
                       vfov_deg=vfov, width=W, height=H)
    return synth.Scene(name="wall", verts=v, tris=t, cache_kind="triangle",
                       cache=np.ones((3, 2), np.float32), emission=np.zeros((3, 2), np.float32),
                       cameras=[cam])


def test_pinhole_geometry():
    for W, H in ((64, 32), (20, 48), (320, 240)):
        sc = _wall_scene(W, H)
        prim = ob.primary(ob.OracleScene(sc))
        P = prim["points"]
        x = P[0].reshape(H, W)
        y = P[1].reshape(H, W)
        z = P[2].reshape(H, W)
        np.testing.assert_allclose(y, 4.0, atol=1e-12)
        dx = np.diff(x, axis=1)
        dz = np.diff(z, axis=0)
        np.testing.assert_allclose(dx, dx[0, 0], rtol=1e-9)
        np.testing.assert_allclose(dz, dz[0, 0], rtol=1e-9)
        assert dx[0, 0] > 0 and dz[0, 0] < 0               # x right, rows downward
        assert abs(dx[0, 0] + dz[0, 0]) < 1e-9 * abs(dx[0, 0])   # square pixels
        # symmetric about the view axis
        np.testing.assert_allclose(x[:, : W // 2], -x[:, ::-1][:, : W // 2], atol=1e-12)
        np.testing.assert_allclose(z[: H // 2], -z[::-1][: H // 2], atol=1e-12)
        # vertical field of view spans the pixel centres of a column
        top = np.array([x[0, 0], 4.0, z[0, 0]])
        bot = np.array([x[-1, 0], 4.0, z[-1, 0]])
        ang_top = math.atan2(top[2], 4.0)
        ang_bot = math.atan2(bot[2], 4.0)
        want = 2 * math.atan(math.tan(math.radians(25.0)) * (1 - 1.0 / H))
        assert abs((ang_top - ang_bot) - want) < 1e-12
        # normal faces the camera, wo points back to it
        np.testing.assert_allclose(P[3:6].T, np.tile([0.0, -1.0, 0.0], (W * H, 1)), atol=1e-15)
        wo = P[6:9]
        pos = P[0:3]
        np.testing.assert_allclose(wo, -pos / np.linalg.norm(pos, axis=0), atol=1e-14)
        assert (prim["tri"] >= 0).all()


def test_tiny_box_points_lie_on_walls(tiny, tiny_points):
    pts, tri, prim = tiny_points
    P = prim["points"]
    V = tiny.verts.astype(np.float64)
    assert (tri >= 0).all()
    for p in range(0, P.shape[1], 7):
        tv = V[tiny.tris[tri[p]]]
        n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
        n /= np.linalg.norm(n)
        # on the triangle's plane, normal parallel to the face normal
        assert abs(np.dot(P[0:3, p] - tv[0], n)) < 1e-12
        assert abs(abs(np.dot(P[3:6, p], n)) - 1.0) < 1e-12
        assert np.dot(P[3:6, p], P[6:9, p]) >= 0.0
