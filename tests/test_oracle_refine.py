"""Pins of the oracle's stage-3 refinement (Sec. 4.3, Eq. 10 and 11).

* With no glossy hit the refinement is the stage-1 bake (Eq. 9 is the
  one-vertex case of Eq. 10): bit for bit when every hit is diffuse, or when
  paths are capped at one vertex, given a zero cache on emitters.
* Two-bounce expectation: on a box with a glossy floor every path ends by
  its second vertex, so a deterministic nested quadrature of Eq. 10 gives
  the value the Monte Carlo refinement estimates; with emitter sampling and
  MIS, and with BRDF sampling only, it must agree within 4 standard errors.
* The BRDF the paths use integrates against the incident radiance to
  kd Ld + ks Ls0 + Ls1 (the factorization of Eq. 5, from the stage-1
  quadrature), and its sampling density integrates to one.
"""
import numpy as np
import pytest

import synth
from oracle import bake as ob

SIGMA_LEVELS = (0.1, 0.5)


def _grid(res=2, sigma=0.9, a=(0.6, 0.4, 0.25), m=0.3):
    g = np.zeros((5, res, res, res), np.float32)
    g[0:3] = np.asarray(a, np.float32)[:, None, None, None]
    g[3] = sigma
    g[4] = m
    return g


def _glossy_floor_grid(sig_floor=0.3, sig_rest=0.9, a=(0.8, 0.5, 0.3), m=0.5, delta=1e-6):
    """A 2-node grid over x, y in [0, 1] and z in [-1, delta]: sigma is
    sig_floor on the plane z = 0 and sig_rest from z = delta on (positions
    above the box clamp onto its top nodes), so only the floor and a strip
    of the walls delta / 2 high are glossy."""
    g = _grid(2, 0.0, a, m)
    v = (sig_floor * (1.0 + delta) - sig_rest) / delta
    g[3, 0] = v          # z = -1 nodes
    g[3, 1] = sig_rest   # z = delta nodes
    return g, (0.0, 0.0, -1.0), (1.0, 1.0, delta)


def _tiny_zero_emitter_cache():
    sc = synth.tiny_box()
    em = sc.emission.max(axis=0) > 0
    sc.cache[:, em] = 0.0
    return sc


@pytest.fixture(scope="module")
def tiny_z():
    sc = _tiny_zero_emitter_cache()
    osc = ob.OracleScene(sc)
    pts, tri = ob.points_f32(ob.primary(osc))
    return sc, osc, pts, tri


def test_all_diffuse_is_the_stage1_bake(tiny_z):
    sc, osc, pts, tri = tiny_z
    idx = np.arange(0, sc.n_points, 5)
    want = ob.bake(osc, pts, tri, idx=idx, spp_d=16, spp_s=8, seed=7)
    got = ob.refine(osc, pts, tri, _grid(sigma=0.9), (0, 0, 0), (1, 1, 1), idx=idx, spp_d=16,
                    spp_s=8, seed=7)
    np.testing.assert_array_equal(got["mean"], want["mean"])


def test_one_vertex_cap_is_the_stage1_bake(tiny_z):
    sc, osc, pts, tri = tiny_z
    idx = np.arange(3, sc.n_points, 7)
    want = ob.bake(osc, pts, tri, idx=idx, spp_d=16, spp_s=8, seed=9)
    got = ob.refine(osc, pts, tri, _grid(sigma=0.2), (0, 0, 0), (1, 1, 1), idx=idx, spp_d=16,
                    spp_s=8, seed=9, max_vertices=1)
    np.testing.assert_array_equal(got["mean"], want["mean"])


def test_all_diffuse_room_per_vertex_cache():
    sc = synth.room(n_cams=1, width=16, height=12)
    em = np.flatnonzero(sc.emission.max(axis=0) > 0)
    sc.cache[:, np.unique(sc.tris[em])] = 0.0       # L' zero on the emitters' vertices
    osc = ob.OracleScene(sc)
    pts, tri = ob.points_f32(ob.primary(osc))
    idx = np.arange(0, sc.n_points, 9)
    want = ob.bake(osc, pts, tri, idx=idx, spp_d=8, spp_s=4, seed=3)
    got = ob.refine(osc, pts, tri, _grid(sigma=0.61), sc.bmin, sc.bmax, idx=idx, spp_d=8, spp_s=4,
                    seed=3)
    np.testing.assert_array_equal(got["mean"], want["mean"])


def _wall_points():
    """A point on the back wall at mid-height and one on the left wall,
    each seen from the tiny box's camera."""
    cam = np.array([0.5, 0.05, 0.5])
    pts = [((0.3, 1.0, 0.45), (0.0, -1.0, 0.0)),
           ((0.0, 0.6, 0.3), (1.0, 0.0, 0.0))]
    P = np.zeros((9, len(pts)), np.float32)
    for q, (x, n) in enumerate(pts):
        wo = cam - np.array(x)
        P[0:3, q], P[3:6, q], P[6:9, q] = x, n, wo / np.linalg.norm(wo)
    return P


SPEC_LEVEL = 0.5


def test_material_lookup_is_trilinear_and_clamped():
    """The refinement's material lookup agrees with the numpy oracle's grid
    gather at random points inside and outside the box, and reproduces an
    affine field exactly."""
    from oracle import render as orr
    rng = np.random.default_rng(4)
    lo, hi = np.array([-0.5, 0.0, 1.0]), np.array([2.0, 1.5, 3.0])
    g = rng.uniform(-1, 1, size=(5, 9, 9, 9)).astype(np.float32)
    x = rng.uniform(-1.0, 3.5, size=(2000, 3))
    got = ob.material_at(g, lo, hi, x)
    want = orr.grid_gather(g, x.T, lo, hi).T
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # affine node values -> the same affine function anywhere in the box
    R = 7
    ax = [lo[a] + np.arange(R) * (hi[a] - lo[a]) / (R - 1) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    A = np.array([[0.5, -0.25, 0.125], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.5, -0.5],
                  [-1.0, 0.0, 2.0]])
    lin = (A[:, 0, None, None, None] * X + A[:, 1, None, None, None] * Y
           + A[:, 2, None, None, None] * Z).astype(np.float32)
    xin = rng.uniform(lo, hi, size=(500, 3))
    got = ob.material_at(lin, lo, hi, xin)
    np.testing.assert_allclose(got, xin @ A.T, rtol=0, atol=2e-6 * np.abs(lin).max())


# A point on the left wall whose narrow specular lobe points down at the
# floor, where the glossy reflection leads to the ceiling emitter: with a
# dark cache the emitter light reflected by the floor dominates its Ls.
MIS_POINT = ((0.0, 0.5, 0.6), (1.0, 0.0, 0.0), (0.298, 0.0, 0.954))
MIS_LEVEL = 0.1


@pytest.fixture(scope="module")
def mis_case():
    sc = _tiny_zero_emitter_cache()
    sc.cache *= 0.02
    osc = ob.OracleScene(sc)
    grid, glo, ghi = _glossy_floor_grid()
    x, n, wo = (np.array(v, np.float64) for v in MIS_POINT)
    wo /= np.linalg.norm(wo)
    P = np.zeros((9, 1), np.float32)
    P[0:3, 0], P[3:6, 0], P[6:9, 0] = x, n, wo
    xd, nd, wd = (P[a:a + 3, 0].astype(np.float64) for a in (0, 3, 6))
    ls, deep = ob.refine_quadrature(osc, xd, nd, wd, 0, grid, glo, ghi,
                                    sigma=float(np.float32(MIS_LEVEL)), n_theta=128, n_phi=128,
                                    n_theta2=48, n_phi2=96)
    assert deep < 1e-5
    return osc, grid, glo, ghi, P, ls


@pytest.mark.parametrize("flags", [0, ob.REFINE_BSDF_ONLY])
def test_emitter_through_glossy_floor_matches_quadrature(mis_case, flags):
    osc, grid, glo, ghi, P, ls = mis_case
    # the floor-reflected emitter dominates: the dark cache alone gives far less
    assert ls[0:3].sum() + ls[3:6].sum() > 0.1
    spp = 16384
    mc = ob.refine(osc, P, np.zeros(1, np.int32), grid, glo, ghi, spp_d=1, spp_s=spp,
                   sigma=(MIS_LEVEL,), seed=33, flags=flags)
    se = ob.std_error(mc, 1, spp)
    z = np.abs(mc["mean"][3:9, 0] - ls) / np.maximum(se[3:9, 0], 1e-12)
    assert np.all(z < 4.0), (mc["mean"][3:9, 0], ls, z)


@pytest.fixture(scope="module")
def two_bounce(tiny_z):
    """Nested quadrature of the refined Ld and of Ls0, Ls1 at one level, at
    the wall points of the box with a glossy floor."""
    sc, osc, _, _ = tiny_z
    grid, glo, ghi = _glossy_floor_grid()
    P = _wall_points()
    sig = float(np.float32(SPEC_LEVEL))
    quad = []
    for q in range(P.shape[1]):
        x, n, wo = (P[a:a + 3, q].astype(np.float64) for a in (0, 3, 6))
        ld, deep_d = ob.refine_quadrature(osc, x, n, wo, -1, grid, glo, ghi, n_theta=96, n_phi=192,
                                          n_theta2=48, n_phi2=96)
        ls, deep_s = ob.refine_quadrature(osc, x, n, wo, 0, grid, glo, ghi, sigma=sig, n_theta=128,
                                          n_phi=192, n_theta2=48, n_phi2=96)
        assert deep_d < 1e-5 and deep_s < 1e-5       # every path ends by its second vertex
        quad.append((ld, ls))
    return sc, osc, grid, glo, ghi, P, quad


@pytest.mark.parametrize("flags", [0, ob.REFINE_BSDF_ONLY])
def test_two_bounce_expectation_matches_quadrature(two_bounce, flags):
    sc, osc, grid, glo, ghi, P, quad = two_bounce
    T = np.zeros(P.shape[1], np.int32)          # any valid triangle index: a surface point
    spp = 16384
    mc = ob.refine(osc, P, T, grid, glo, ghi, spp_d=spp, spp_s=spp, sigma=(SPEC_LEVEL,), seed=21,
                   flags=flags)
    se = ob.std_error(mc, spp, spp)
    for q, (ld, ls) in enumerate(quad):
        z = np.abs(mc["mean"][0:3, q] - ld) / se[0:3, q]
        assert np.all(z < 4.0), (q, "Ld", mc["mean"][0:3, q], ld, z)
        got = mc["mean"][3:9, q]
        z = np.abs(got - ls) / np.maximum(se[3:9, q], 1e-12)
        assert np.all(z < 4.0), (q, "Ls", got, ls, z)


def test_two_bounce_differs_from_stage1(two_bounce):
    """The glossy floor matters: the refined expectation differs from the
    stage-1 integral of the cache (both by deterministic quadrature)."""
    sc, osc, grid, glo, ghi, P, quad = two_bounce
    for q, (ld, ls) in enumerate(quad):
        x, n, wo = (P[a:a + 3, q].astype(np.float64) for a in (0, 3, 6))
        ld1 = ob.quadrature(osc, x, n, wo, -1, n_theta=96, n_phi=192)
        assert np.max(np.abs(ld - ld1) / ld1) > 0.02, (q, ld, ld1)


def test_brdf_integrates_to_the_factorized_render(tiny_z):
    """At a floor point with sigma equal to a level, integrating f of Eq. 1
    against the incident radiance gives kd Ld + ks Ls0 + Ls1 (Eq. 5), each
    shading from the stage-1 quadrature."""
    sc, osc, _, _ = tiny_z
    x = np.array([0.4, 0.55, 0.0])
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.1, -0.5, 0.8])
    wo /= np.linalg.norm(wo)
    a = np.array([0.7, 0.4, 0.2])
    m, sig = 0.3, 0.5
    Ld = ob.quadrature(osc, x, n, wo, -1, n_theta=256, n_phi=512)
    Ls = ob.quadrature(osc, x, n, wo, 0, sigma=sig, n_theta=256, n_phi=512)
    kd, ks = a * (1 - m), 0.04 * (1 - m) + a * m
    want = kd * Ld + ks * Ls[:3] + Ls[3:]
    # midpoint rule over the hemisphere with f evaluated by the oracle
    nt, nph = 256, 512
    th = (np.arange(nt) + 0.5) * (0.5 * np.pi / nt)
    ph = (np.arange(nph) + 0.5) * (2 * np.pi / nph)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    t, b = ob.frame(n)
    loc = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    wi = loc[:, 0:1] * t + loc[:, 1:2] * b + loc[:, 2:3] * n
    Li = ob.trace_radiance(osc, np.tile(x + 1e-4 * n, (len(wi), 1)), wi)
    f = np.array([ob.brdf(n, wo, w, a, sig, m) for w in wi])
    dw = (np.sin(TH) * (0.5 * np.pi / nt) * (2 * np.pi / nph)).reshape(-1, 1)
    got = (f * Li * dw).sum(0)
    np.testing.assert_allclose(got, want, rtol=4e-3)


@pytest.mark.parametrize("sig", [0.1, 0.35, 0.6])
def test_sampling_density_integrates_to_one(sig):
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.3, 0.2, 0.9])
    wo /= np.linalg.norm(wo)
    # over half vectors (stretched near the lobe), d omega_i = 4 (wo.h) d omega_h
    nt, nph = 512, 256
    s = (np.arange(nt) + 0.5) / nt
    th = 0.5 * np.pi * s ** 4
    dth = 0.5 * np.pi * 4 * s ** 3 / nt
    ph = (np.arange(nph) + 0.5) * (2 * np.pi / nph)
    total = 0.0
    for i in range(nt):
        h = np.stack([np.sin(th[i]) * np.cos(ph), np.sin(th[i]) * np.sin(ph),
                      np.full(nph, np.cos(th[i]))], -1)
        oh = h @ wo
        wi = 2 * oh[:, None] * h - wo
        ok = (oh > 0) & (wi[:, 2] > 0)
        # only the GGX half of the mixture: its density in h is D(h)(n.h) / 2
        pdf_i = np.array([ob.brdf_pdf(n, wo, w, sig) if k else 0.0 for w, k in zip(wi, ok)])
        cos_pdf = np.where(ok, 0.5 * wi[:, 2] / np.pi, 0.0)
        total += np.sum((pdf_i - cos_pdf) * 4 * np.maximum(oh, 0) * np.sin(th[i]) * dth[i]
                        * (2 * np.pi / nph))
    # GGX half: 1/2 less what reflects below the horizon (nothing at a
    # narrow lobe around a near-normal view); the cosine half: exactly 1/2
    assert total <= 0.5 + 1e-3
    if sig <= 0.1:
        assert total >= 0.5 - 2e-3
    # the full mixture over wi directly
    nt2 = 256
    th2 = (np.arange(nt2) + 0.5) * (0.5 * np.pi / nt2)
    acc = 0.0
    for i in range(nt2):
        wi = np.stack([np.sin(th2[i]) * np.cos(ph), np.sin(th2[i]) * np.sin(ph),
                       np.full(nph, np.cos(th2[i]))], -1)
        pdf = np.array([ob.brdf_pdf(n, wo, w, sig) for w in wi])
        acc += pdf.sum() * np.sin(th2[i]) * (0.5 * np.pi / nt2) * (2 * np.pi / nph)
    assert abs(acc - (0.5 + total)) < 2e-2 * (1 if sig < 0.2 else 0.25)


def test_envelope_and_arguments(tiny_z):
    sc, osc, pts, tri = tiny_z
    grid, glo, ghi = _glossy_floor_grid()
    idx = np.arange(0, sc.n_points, 3)
    r = ob.refine(osc, pts, tri, grid, glo, ghi, idx=idx, spp_d=32, spp_s=16, seed=5)
    assert np.all(r["lo"] <= r["mean"] + 1e-12) and np.all(r["mean"] <= r["hi"] + 1e-12)
    assert r["n_ambiguous"] > 0      # pixel-centre points on shared edges, paths grazing them
    with pytest.raises(ValueError):
        ob.refine(osc, pts, tri, grid, glo, ghi, idx=idx[:4], max_vertices=0)
    with pytest.raises(ValueError):
        ob.refine(osc, pts, tri, grid, glo, ghi, idx=idx[:4], max_vertices=17)
