"""Pins of the oracle's microfacet pieces (the BRDF of Eq. 1 and the
sampling used for Eq. 6) against closed forms:

* GGX D integrates to one over projected half vectors, for every level;
* Smith G1 paired with GGX D satisfies the weak white furnace identity
  (Heitz 2014): the integral of G1(wo) max(0, wo.m) D(m) over m equals n.wo;
* the GGX sampler draws theta_m with the density D(m) cos(theta_m);
* the cosine sampler has E[cos] = 2/3, E[cos^2] = 1/2;
* the frame is orthonormal and right-handed for every normal.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import bake as ob

SIGMAS = (0.02, 0.1, 0.25, 0.5, 0.75, 1.0)


def _theta_integral(f, alpha):
    pts = [p for p in (alpha, 3 * alpha, 10 * alpha, 30 * alpha) if p < math.pi / 2]
    val, err = integrate.quad(f, 0.0, math.pi / 2, points=pts, limit=500,
                              epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("sigma", SIGMAS)
def test_ggx_D_normalised(sigma):
    alpha = sigma * sigma
    val = 2 * math.pi * _theta_integral(
        lambda th: ob.ggx_D(alpha, math.cos(th)) * math.cos(th) * math.sin(th), alpha)
    assert abs(val - 1.0) < 1e-7


def _phi_integral(A, B):
    """Integral over phi in [0, 2pi) of max(0, A cos(phi) + B), A >= 0."""
    if B >= A:
        return 2 * math.pi * B
    if B <= -A:
        return 0.0
    p0 = math.acos(-B / A)
    return 2 * (A * math.sin(p0) + B * p0)


@pytest.mark.parametrize("sigma", SIGMAS)
@pytest.mark.parametrize("theta_o_deg", [0.0, 30.0, 60.0, 80.0, 89.0])
def test_weak_white_furnace_identity(sigma, theta_o_deg):
    alpha = sigma * sigma
    to = math.radians(theta_o_deg)
    co, so = math.cos(to), math.sin(to)

    def f(th):
        A = so * math.sin(th)
        B = co * math.cos(th)
        return ob.ggx_D(alpha, math.cos(th)) * math.sin(th) * _phi_integral(A, B)

    val = ob.ggx_G1(alpha, co) * _theta_integral(f, alpha)
    assert abs(val - co) < 1e-6 * max(co, 1e-3) + 1e-9


def test_G1_limits():
    for a in (1e-4, 0.01, 0.25, 1.0):
        assert ob.ggx_G1(a, 1.0) == 1.0
        assert ob.ggx_G1(a, 1e-9) < 1e-6 / a + 1e-6
        prev = 0.0
        for c in np.linspace(0.01, 1.0, 50):
            g = ob.ggx_G1(a, c)
            assert 0.0 < g <= 1.0 and g >= prev
            prev = g
    assert abs(ob.ggx_G1(1e-8, 0.05) - 1.0) < 1e-9
    assert ob.ggx_G1(0.5, -0.1) == 0.0


@pytest.mark.parametrize("sigma", (0.1, 0.5, 1.0))
def test_ggx_sampler_density(sigma):
    """Kolmogorov-Smirnov of sampled theta_m against the CDF obtained by
    integrating D(m) cos(theta_m) with the oracle's D (not its sampler)."""
    alpha = sigma * sigma
    rng = np.random.default_rng(3)
    n = 20000
    xi = rng.random((n, 2))
    th = np.array([math.acos(min(1.0, ob.sample_ggx(alpha, a, b)[2])) for a, b in xi])
    grid = np.linspace(0, math.pi / 2, 4001)
    dens = np.array([2 * math.pi * ob.ggx_D(alpha, math.cos(t)) * math.cos(t) * math.sin(t)
                     for t in grid])
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    d, p = stats.kstest(th, lambda x: np.interp(x, grid, cdf))
    assert p > 1e-3
    # azimuth uniform
    ph = np.array([math.atan2(*ob.sample_ggx(alpha, a, b)[[1, 0]]) for a, b in xi[:5000]])
    assert stats.kstest((ph + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3


def test_cosine_sampler_moments():
    rng = np.random.default_rng(4)
    xi = rng.random((40000, 2))
    d = np.array([ob.sample_cosine(a, b) for a, b in xi])
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    se = 1.0 / math.sqrt(len(d))
    assert abs(d[:, 2].mean() - 2.0 / 3.0) < 5 * se * 0.24
    assert abs((d[:, 2] ** 2).mean() - 0.5) < 5 * se * 0.29
    assert abs(d[:, 0].mean()) < 5 * se * 0.5 and abs(d[:, 1].mean()) < 5 * se * 0.5
    assert d[:, 2].min() > 0.0


def test_frame_orthonormal():
    rng = np.random.default_rng(5)
    ns = [np.array(v, float) for v in ((0, 0, 1), (0, 0, -1), (1, 0, 0), (0, 1, 0),
                                       (-1, 0, 0), (0, -1, 0), (0, 1, -0.0))]
    for v in rng.standard_normal((200, 3)):
        ns.append(v / np.linalg.norm(v))
    for n in ns:
        t, b = ob.frame(n)
        M = np.stack([t, b, n])
        np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(np.cross(t, b), n, atol=1e-12)
