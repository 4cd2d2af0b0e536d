"""Pins of the oracle's factored re-render, loss and gradient (Eq. 5, 8, 2,
15) and of the trilinear material grid:

* at a tabulated roughness the render reproduces that level exactly;
* kd and ks reach their defining limits at m = 0 and m = 1;
* the loss is a quadratic in (a, m) for fixed roughness, so central finite
  differences in float64 equal the analytic gradient to rounding; the same
  holds for roughness inside one interpolation segment;
* an independent torch float64 autograd expression agrees;
* the grid reproduces any affine function exactly and its adjoint satisfies
  <gather(G), p> = <G, scatter(p)>.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import render as orr

SIG = np.array(synth.SIGMA_GRID)


def _inputs(n=257, seed=0):
    sh = synth.random_shading(n, 6, seed=seed).astype(np.float64)
    mat = synth.random_materials(n, seed=seed + 1).astype(np.float64)
    gt = synth.random_observations(n, seed=seed + 2).astype(np.float64)
    return sh, mat, gt


def test_render_at_knots_reproduces_levels():
    sh, mat, _ = _inputs()
    K = 6
    for k in range(K):
        m = mat.copy()
        m[3] = SIG[k]
        Lr = orr.render(sh, m, SIG)["Lr"]
        a, met = m[0:3], m[4]
        kd = a * (1 - met)
        ks = 0.04 * (1 - met) + a * met
        Ld = sh[0:3]
        L0 = sh[3 + 3 * k:6 + 3 * k]
        L1 = sh[3 + 3 * K + 3 * k:6 + 3 * K + 3 * k]
        np.testing.assert_array_equal(Lr, kd * Ld + ks * L0 + L1)


def test_reflectance_limits():
    sh, mat, _ = _inputs()
    K = 6
    Ld = sh[0:3]
    m0 = mat.copy()
    m0[4] = 0.0
    m0[3] = SIG[2]
    r0 = orr.render(sh, m0, SIG)
    # m = 0: kd = a, ks = 0.04
    np.testing.assert_allclose(r0["Lr"], m0[0:3] * Ld + 0.04 * sh[9:12] + sh[3 + 3 * K + 6:3 + 3 * K + 9],
                               rtol=1e-15)
    m1 = m0.copy()
    m1[4] = 1.0
    r1 = orr.render(sh, m1, SIG)
    # m = 1: kd = 0, ks = a
    np.testing.assert_allclose(r1["Lr"], m1[0:3] * sh[9:12] + sh[3 + 3 * K + 6:3 + 3 * K + 9], rtol=1e-15)


def test_interpolation_is_linear_between_knots():
    sh, mat, _ = _inputs()
    K = 6
    m = mat.copy()
    m[4] = 0.3
    lo, hi = SIG[3], SIG[4]
    m[3] = lo
    A = orr.render(sh, m, SIG)["Lr"]
    m[3] = hi
    B = orr.render(sh, m, SIG)["Lr"]
    for t in (0.25, 0.5, 0.9):
        m[3] = lo + t * (hi - lo)
        np.testing.assert_allclose(orr.render(sh, m, SIG)["Lr"], (1 - t) * A + t * B, rtol=1e-12, atol=1e-14)
    # clamped outside the grid
    m[3] = 0.0
    np.testing.assert_allclose(orr.render(sh, m, SIG)["Lr"],
                               orr.render(sh, np.where(np.arange(5)[:, None] == 3, SIG[0], m), SIG)["Lr"])
    m[3] = 1.7
    np.testing.assert_allclose(orr.render(sh, m, SIG)["Lr"],
                               orr.render(sh, np.where(np.arange(5)[:, None] == 3, SIG[-1], m), SIG)["Lr"])


@pytest.mark.parametrize("tone", [0, 1])
def test_gradient_central_differences(tone):
    sh, mat, gt = _inputs(n=64, seed=3)
    # keep roughness away from the knots so sigma +- eps stays in one segment
    j, t, cl = orr.bracket(SIG, mat[3])
    away = (np.abs(mat[3][:, None] - SIG[None, :]).min(axis=1) > 2e-3)
    mat = mat[:, away]
    sh = sh[:, away]
    gt = gt[:, away]
    loss, grad, _ = orr.loss_and_grad(sh, mat, gt, SIG, tone)
    eps = 1e-3 if tone == 0 else 1e-5
    for c in range(5):
        for p in range(mat.shape[1]):
            mp, mm = mat.copy(), mat.copy()
            mp[c, p] += eps
            mm[c, p] -= eps
            fd = (orr.loss_and_grad(sh, mp, gt, SIG, tone)[0]
                  - orr.loss_and_grad(sh, mm, gt, SIG, tone)[0]) / (2 * eps)
            tol = 1e-9 * max(1.0, abs(loss)) if tone == 0 else 1e-6 * max(1.0, abs(fd))
            assert abs(fd - grad[c, p]) < tol, (c, p, fd, grad[c, p])


def test_gradient_matches_torch_autograd():
    """Third opinion: torch float64 autograd of an independently written
    expression of the same loss (per-point lerp by explicit masks)."""
    sh, mat, gt = _inputs(n=300, seed=5)
    loss, grad, Lr = orr.loss_and_grad(sh, mat, gt, SIG, 0)
    K = 6
    S = torch.tensor(sh)
    M = torch.tensor(mat, requires_grad=True)
    G = torch.tensor(gt)
    sig = torch.tensor(SIG)
    a, s, m = M[0:3], M[3], M[4]
    sc = torch.clamp(s, sig[0], sig[-1])
    L0 = torch.zeros(3, S.shape[1], dtype=torch.float64)
    L1 = torch.zeros_like(L0)
    for k in range(K - 1):
        last = k == K - 2
        inseg = (sc >= sig[k]) & ((sc < sig[k + 1]) | torch.tensor(last))
        w = (sc - sig[k]) / (sig[k + 1] - sig[k])
        seg0 = (1 - w) * S[3 + 3 * k:6 + 3 * k] + w * S[6 + 3 * k:9 + 3 * k]
        seg1 = (1 - w) * S[3 + 3 * K + 3 * k:6 + 3 * K + 3 * k] + w * S[6 + 3 * K + 3 * k:9 + 3 * K + 3 * k]
        L0 = torch.where(inseg, seg0, L0)
        L1 = torch.where(inseg, seg1, L1)
    out = a * (1 - m) * S[0:3] + (0.04 * (1 - m) + a * m) * L0 + L1
    l = ((out - G) ** 2).sum()
    l.backward()
    np.testing.assert_allclose(l.item(), loss, rtol=1e-13)
    np.testing.assert_allclose(out.detach().numpy(), Lr, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(M.grad.numpy(), grad, rtol=1e-11, atol=1e-13)


def test_tonemap_derivative():
    x = np.linspace(-0.5, 60.0, 2001)
    x = x[np.abs(np.expm1(0.0031308) - x) > 1e-4]
    h = 1e-6
    fd = (orr.tonemap(x + h, 1) - orr.tonemap(x - h, 1)) / (2 * h)
    mask = np.abs(x) > 2e-6
    np.testing.assert_allclose(orr.tonemap_d(x, 1)[mask], fd[mask], rtol=1e-6, atol=1e-8)
    assert orr.tonemap(0.0, 1) == 0.0
    assert abs(orr.tonemap(math.e - 1.0, 1) - 1.0) < 1e-12   # log(1 + x) = 1 -> sRGB(1) = 1


def test_grid_affine_exact_and_adjoint():
    rng = np.random.default_rng(2)
    R = 9
    bmin = np.array([-1.0, 0.5, 2.0])
    bmax = np.array([3.0, 2.5, 7.0])
    nodes = [bmin[d] + np.arange(R) * (bmax[d] - bmin[d]) / (R - 1) for d in range(3)]
    Z, Y, X = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    coef = rng.standard_normal((5, 4))
    grid = np.stack([c[0] * X + c[1] * Y + c[2] * Z + c[3] for c in coef])
    x = np.stack([rng.uniform(bmin[d], bmax[d], 500) for d in range(3)])
    got = orr.grid_gather(grid, x, bmin, bmax)
    want = np.stack([c[0] * x[0] + c[1] * x[1] + c[2] * x[2] + c[3] for c in coef])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # node positions return node values; outside points clamp onto the box
    xn = np.array([[nodes[0][3]], [nodes[1][0]], [nodes[2][8]]])
    np.testing.assert_allclose(orr.grid_gather(grid, xn, bmin, bmax)[:, 0], grid[:, 8, 0, 3], rtol=1e-12)
    xo = np.array([[bmax[0] + 5.0], [bmin[1] - 1.0], [bmin[2] + 0.0]])
    np.testing.assert_allclose(orr.grid_gather(grid, xo, bmin, bmax)[:, 0], grid[:, 0, 0, R - 1], rtol=1e-12)
    # adjoint identity
    G = rng.standard_normal((5, R, R, R))
    P = rng.standard_normal((5, 500))
    lhs = np.sum(orr.grid_gather(G, x, bmin, bmax) * P)
    rhs = np.sum(G * orr.grid_scatter(P, x, bmin, bmax, R))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))
