"""Pins of the oracle's Monte Carlo bake (Eq. 6, 7, 9) against closed forms
and an independent deterministic quadrature.

* furnace: a closed box whose cache is the constant L everywhere returns
  Ld = L exactly (zero-variance estimator), so pi * Ld equals the
  irradiance pi * L;
* the specular terms in the same box: Ls0 + Ls1 never exceeds L in
  expectation (energy conservation of the GGX-Smith lobe) and tends to L
  as roughness goes to zero;
* weak white furnace (Heitz 2014): with G replaced by G1(wo), no horizon
  clipping and unit radiance, E[Ls0 + Ls1] = 1 for every view angle;
* Lambert's polygon formula for the irradiance from a uniform polygonal
  emitter: pi * Ld at unoccluded points equals it;
* quadrature: each lobe's integral at a handful of points equals the Monte
  Carlo estimate within its standard error;
* results depend only on the point index (batching independence).
"""
import copy
import math

import numpy as np
import pytest

import synth
from oracle import bake as ob


def _clean(res):
    """Points whose samples are all unambiguous (lo == hi everywhere)."""
    return np.all(res["hi"] - res["lo"] == 0.0, axis=0)


def test_furnace_diffuse_exact(tiny, tiny_points):
    pts, tri, _ = tiny_points
    sc = copy.deepcopy(tiny)
    L = np.float32(0.7)
    sc.cache[:] = L
    sc.emission[:] = 0
    osc = ob.OracleScene(sc)
    r = ob.bake(osc, pts, tri, spp_d=64, spp_s=8, seed=sc.seed)
    valid = tri >= 0
    clean = _clean(r) & valid
    assert clean.sum() > 4000
    np.testing.assert_allclose(r["mean"][0:3, clean], float(L), rtol=1e-14)
    np.testing.assert_allclose(math.pi * r["mean"][0:3, clean], math.pi * float(L), rtol=1e-14)
    # degenerate points (exactly on a box edge) still bracket L
    amb = valid & ~clean
    assert np.all(r["lo"][0:3, amb] <= L + 1e-12) and np.all(r["hi"][0:3, amb] >= L - 1e-12)


def test_furnace_specular_bounded(tiny, tiny_points):
    pts, tri, _ = tiny_points
    sc = copy.deepcopy(tiny)
    sc.cache[:] = 1.0
    sc.emission[:] = 0
    osc = ob.OracleScene(sc)
    _, _, prim = tiny_points
    idx = np.arange(0, 4096, 97)
    idx = idx[(tri[idx] >= 0) & (prim["n_outcomes"][idx] == 1)]
    spp = 2048
    r = ob.bake(osc, pts, tri, idx=idx, spp_d=1, spp_s=spp, seed=sc.seed)
    K = 6
    tot = r["mean"][3:3 + 3 * K].reshape(K, 3, -1) + r["mean"][3 + 3 * K:].reshape(K, 3, -1)
    # standard error of the sum from its own second moment is not tracked;
    # bound each term's SE and add them
    se = ob.std_error(r, 1, spp)
    se_tot = se[3:3 + 3 * K].reshape(K, 3, -1) + se[3 + 3 * K:].reshape(K, 3, -1)
    assert np.all(tot <= 1.0 + 5 * se_tot + 1e-12)
    assert np.all(tot > 0.0)
    mean_per_level = tot[:, 0].mean(axis=1)
    assert np.all(np.diff(mean_per_level) < 0.0)        # rougher reflects less
    assert mean_per_level[0] > 0.98                      # near-mirror keeps almost all


@pytest.mark.parametrize("theta_deg", [0.0, 40.0, 75.0, 88.0])
def test_weak_white_furnace_mc(theta_deg):
    """A single upward-facing point with wo at theta from the normal; unit
    radiance for every sample; G replaced by G1(wo)."""
    sc = synth.tiny_box()
    osc = ob.OracleScene(sc)
    th = math.radians(theta_deg)
    pts = np.zeros((9, 1), np.float32)
    pts[0:3, 0] = (0.5, 0.5, 0.0)
    pts[3:6, 0] = (0.0, 0.0, 1.0)
    pts[6:9, 0] = (math.sin(th), 0.0, math.cos(th))
    tri = np.zeros(1, np.int32)
    spp = 1 << 16
    r = ob.bake(osc, pts, tri, spp_d=1, spp_s=spp, seed=99, flags=ob.WEAK_FURNACE)
    K = 6
    s0 = r["mean"][3:3 + 3 * K:3, 0]
    s1 = r["mean"][3 + 3 * K::3, 0]
    se = ob.std_error(r, 1, spp)
    bound = se[3:3 + 3 * K:3, 0] + se[3 + 3 * K::3, 0]
    np.testing.assert_array_less(np.abs(s0 + s1 - 1.0), 4.0 * bound + 1e-12)


def _polygon_irradiance(x, n, poly, L):
    """Lambert's formula: irradiance at x (normal n) from a uniform polygon
    of radiance L = (L/2) * |sum_k beta_k (gamma_k . n)|."""
    r = [(p - x) / np.linalg.norm(p - x) for p in poly]
    s = 0.0
    for k in range(len(r)):
        a, b = r[k], r[(k + 1) % len(r)]
        beta = math.acos(np.clip(np.dot(a, b), -1.0, 1.0))
        g = np.cross(a, b)
        g /= np.linalg.norm(g)
        s += beta * np.dot(g, n)
    return 0.5 * L * abs(s)


def test_plane_irradiance_lambert(tiny, tiny_points):
    pts, tri, _ = tiny_points
    sc = copy.deepcopy(tiny)
    sc.cache[:] = 0.0     # only the ceiling emitter lights the room
    osc = ob.OracleScene(sc)
    on_floor = np.where((tri >= 0) & (tri <= 1))[0]
    on_wall = np.where((tri >= 2) & (tri <= 9))[0]
    idx = np.concatenate([on_floor[:: max(1, len(on_floor) // 6)][:6],
                          on_wall[:: max(1, len(on_wall) // 6)][:6]])
    spp = 1 << 15
    r = ob.bake(osc, pts, tri, idx=idx, spp_d=spp, spp_s=1, seed=7)
    se = ob.std_error(r, spp, 1)
    poly = [np.array(v, float) for v in ((0.375, 0.375, 1), (0.625, 0.375, 1),
                                         (0.625, 0.625, 1), (0.375, 0.625, 1))]
    for q, p in enumerate(idx):
        x = pts[0:3, p].astype(np.float64)
        n = pts[3:6, p].astype(np.float64)
        E = _polygon_irradiance(x, n, poly, 10.0)
        got = math.pi * r["mean"][0, q]
        assert abs(got - E) < 4.5 * math.pi * se[0, q] + 1e-9, (p, got, E)


def test_quadrature_matches_monte_carlo(tiny, tiny_oracle, tiny_points):
    """Eq. 6 integrals evaluated two ways at 6 points of the tiny box (random
    per-triangle cache plus the emitter): the deterministic quadrature and
    the importance-sampled Monte Carlo estimate."""
    pts, tri, prim = tiny_points
    rng = np.random.default_rng(17)
    cand = np.where((tri >= 0) & (prim["n_outcomes"] == 1))[0]
    idx = np.sort(rng.choice(cand, 6, replace=False))
    spp = 1 << 14
    r = ob.bake(tiny_oracle, pts, tri, idx=idx, spp_d=spp, spp_s=spp, seed=31)
    se = ob.std_error(r, spp, spp)
    K = len(tiny.sigma)
    for q, p in enumerate(idx):
        x = pts[0:3, p].astype(np.float64)
        n = pts[3:6, p].astype(np.float64)
        wo = pts[6:9, p].astype(np.float64)
        qd = ob.quadrature(tiny_oracle, x, n, wo, -1, n_theta=400, n_phi=800)
        for c in range(3):
            assert abs(qd[c] - r["mean"][c, q]) < 4.5 * se[c, q] + 3e-3 * abs(qd[c]) + 1e-9
        for k, s in enumerate(tiny.sigma):
            qs = ob.quadrature(tiny_oracle, x, n, wo, 0, sigma=s, n_theta=600, n_phi=600)
            for c in range(3):
                j0, j1 = 3 + 3 * k + c, 3 + 3 * K + 3 * k + c
                # the Fresnel part F1 = (1 - wi.m)^5 of a narrow lobe seen near
                # the normal is carried by rare far-tail half vectors, where the
                # sample variance understates the error: floor of 1e-6 of the
                # lobe's total (Ls0 + Ls1) on both parts
                floor = 1e-6 * (abs(qs[c]) + abs(qs[3 + c])) + 1e-9
                assert abs(qs[c] - r["mean"][j0, q]) < 4.5 * se[j0, q] + 3e-3 * abs(qs[c]) + floor, (p, s, c)
                assert abs(qs[3 + c] - r["mean"][j1, q]) < 4.5 * se[j1, q] + 3e-3 * abs(qs[3 + c]) + floor, (p, s, c)


def test_deterministic_and_batch_independent(tiny_oracle, tiny_points):
    pts, tri, _ = tiny_points
    full = ob.bake(tiny_oracle, pts, tri, spp_d=16, spp_s=16, seed=5)
    again = ob.bake(tiny_oracle, pts, tri, spp_d=16, spp_s=16, seed=5, threads=3)
    np.testing.assert_array_equal(full["mean"], again["mean"])
    sub = np.array([4095, 7, 1000, 7])
    part = ob.bake(tiny_oracle, pts, tri, idx=sub, spp_d=16, spp_s=16, seed=5)
    np.testing.assert_array_equal(part["mean"], full["mean"][:, sub])
    assert np.all(full["lo"] <= full["mean"]) and np.all(full["mean"] <= full["hi"])
    other = ob.bake(tiny_oracle, pts, tri, spp_d=16, spp_s=16, seed=6)
    assert np.any(other["mean"] != full["mean"])
