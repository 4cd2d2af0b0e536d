"""Pins of the oracle's emission-masked loss (Eq. 12 / 15) and diffuse prior
(Eq. 17):

* with alpha = 0 and no prior it is the plain loss of Eq. 2 / 15 (itself
  pinned in the render tests), and d loss / d alpha has the closed form
  -2 sum_c (Lr - Lgt)^2 under the identity tone map;
* with a uniform alpha and the identity tone map the masked residual is
  (1 - alpha) times the plain one, so loss and material gradient scale by
  (1 - alpha)^2 and d loss / d alpha = -2 (1 - alpha) sum_c (Lr - Lgt)^2;
* alpha = 1 removes the photometric term: only the prior is left;
* a perfect fit leaves the prior alone, with hand-computed values, and the
  sign(0) = 0 reading at sigma = 1, m = 0;
* central finite differences of the total in alpha and in every material
  channel, under both tone maps, and torch float64 autograd of an
  independently written expression agree with the analytic gradients.
"""
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


@pytest.mark.parametrize("tone", [0, 1])
def test_zero_mask_no_prior_is_plain_loss(tone):
    sh, mat, gt = _inputs(seed=1)
    n = mat.shape[1]
    loss, grad, ga, lr = orr.masked_loss_and_grad(sh, mat, gt, np.zeros(n), SIG, tone, 0.0)
    l0, g0, lr0 = orr.loss_and_grad(sh, mat, gt, SIG, tone)
    assert loss == l0
    np.testing.assert_array_equal(grad, g0)
    np.testing.assert_array_equal(lr, lr0)
    if tone == 0:
        np.testing.assert_allclose(ga, -2.0 * np.sum((lr0 - gt) ** 2, axis=0), rtol=1e-13)


@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.9])
def test_uniform_mask_scales_the_residual(alpha):
    sh, mat, gt = _inputs(seed=2)
    n = mat.shape[1]
    loss, grad, ga, lr = orr.masked_loss_and_grad(sh, mat, gt, np.full(n, alpha), SIG, 0, 0.0)
    l0, g0, lr0 = orr.loss_and_grad(sh, mat, gt, SIG, 0)
    f = (1.0 - alpha) ** 2
    np.testing.assert_allclose(loss, f * l0, rtol=1e-12)
    np.testing.assert_allclose(grad, f * g0, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(ga, -2.0 * (1.0 - alpha) * np.sum((lr0 - gt) ** 2, axis=0),
                               rtol=1e-10)
    np.testing.assert_array_equal(lr, lr0)


@pytest.mark.parametrize("tone", [0, 1])
def test_full_mask_leaves_only_the_prior(tone):
    sh, mat, gt = _inputs(seed=3)
    n = mat.shape[1]
    lam = 5e-4
    rng = np.random.default_rng(31)
    mat[3] = rng.uniform(0.01, 0.99, n)
    mat[4] = rng.uniform(0.01, 0.99, n)
    loss, grad, ga, _ = orr.masked_loss_and_grad(sh, mat, gt, np.ones(n), SIG, tone, lam)
    np.testing.assert_allclose(loss, lam * np.sum((1.0 - mat[3]) + mat[4]), rtol=1e-13)
    np.testing.assert_array_equal(grad[0:3], 0.0)
    np.testing.assert_array_equal(grad[3], -lam)
    np.testing.assert_array_equal(grad[4], lam)
    np.testing.assert_array_equal(ga, 0.0)


def test_perfect_fit_hand_values():
    sh, mat, _ = _inputs(n=40, seed=4)
    mat[3] = 0.25
    mat[4] = 0.5
    mat[3, :5] = 1.0      # |1 - sigma| at its kink
    mat[4, 5:10] = 0.0    # |m| at its kink
    gt = orr.render(sh, mat, SIG)["Lr"]
    rng = np.random.default_rng(5)
    alpha = rng.uniform(0, 1, 40)
    lam = 2.0
    loss, grad, ga, _ = orr.masked_loss_and_grad(sh, mat, gt, alpha, SIG, 1, lam)
    # 5 points with sigma = 1 (prior 0 + 0.5), 5 with m = 0 (0.75 + 0), 30 with 1.25
    assert loss == pytest.approx(lam * (5 * 0.5 + 5 * 0.75 + 30 * 1.25), rel=1e-14)
    # at a perfect fit the photometric gradient vanishes up to the rounding
    # of (1 - alpha) Lgt + alpha Lgt; sigma = 1 is clamped at the top knot
    np.testing.assert_allclose(grad[0:3], 0.0, atol=1e-14)
    want_s = np.full(40, -lam)
    want_s[:5] = 0.0
    want_m = np.full(40, lam)
    want_m[5:10] = 0.0
    np.testing.assert_allclose(grad[3], want_s, rtol=0, atol=1e-14)
    np.testing.assert_allclose(grad[4], want_m, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ga, 0.0, atol=1e-14)


@pytest.mark.parametrize("tone", [0, 1])
def test_central_differences(tone):
    sh, mat, gt = _inputs(n=48, seed=6)
    away = np.abs(mat[3][:, None] - SIG[None, :]).min(axis=1) > 2e-3
    away &= mat[4] > 2e-3
    sh, mat, gt = sh[:, away], mat[:, away], gt[:, away]
    n = mat.shape[1]
    alpha = np.random.default_rng(7).uniform(0.05, 0.95, n)
    lam = 0.3
    loss, grad, ga, _ = orr.masked_loss_and_grad(sh, mat, gt, alpha, SIG, tone, lam)
    eps = 1e-3 if tone == 0 else 1e-5

    def total(m, a):
        return orr.masked_loss_and_grad(sh, m, gt, a, SIG, tone, lam)[0]

    for p in range(n):
        ap, am = alpha.copy(), alpha.copy()
        ap[p] += eps
        am[p] -= eps
        fd = (total(mat, ap) - total(mat, am)) / (2 * eps)
        tol = 1e-9 * max(1.0, abs(loss)) if tone == 0 else 1e-6 * max(1.0, abs(fd))
        assert abs(fd - ga[p]) < tol, (p, fd, ga[p])
        for c in range(5):
            mp, mm = mat.copy(), mat.copy()
            mp[c, p] += eps
            mm[c, p] -= eps
            fd = (total(mp, alpha) - total(mm, alpha)) / (2 * eps)
            assert abs(fd - grad[c, p]) < tol, (c, p, fd, grad[c, p])


def test_matches_torch_autograd_with_tonemap():
    """torch float64 autograd of an independently written expression
    (explicit segment masks, tone map written out) for loss, material and
    mask gradients."""
    sh, mat, gt = _inputs(n=300, seed=8)
    rng = np.random.default_rng(9)
    alpha = rng.uniform(0, 1, 300)
    alpha[:10] = 0.0
    alpha[10:20] = 1.0
    lam = 5e-4
    loss, grad, ga, _ = orr.masked_loss_and_grad(sh, mat, gt, alpha, SIG, 1, lam)
    K = 6
    S = torch.tensor(sh)
    M = torch.tensor(mat, requires_grad=True)
    A = torch.tensor(alpha, requires_grad=True)
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
    Lr = a * (1 - m) * S[0:3] + (0.04 * (1 - m) + a * m) * L0 + L1

    def gamma(x):
        y = torch.log1p(torch.clamp(x, min=0.0))
        lin = 12.92 * y
        pw = 1.055 * torch.pow(torch.clamp(y, min=0.0031308), 1 / 2.4) - 0.055
        return torch.where(y <= 0.0031308, lin, pw)

    Lhat = (1 - A) * Lr + A * G
    l = ((gamma(Lhat) - gamma(G)) ** 2).sum() + lam * (torch.abs(1 - s) + torch.abs(m)).sum()
    l.backward()
    np.testing.assert_allclose(l.item(), loss, rtol=1e-12)
    np.testing.assert_allclose(A.grad.numpy(), ga, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(M.grad.numpy(), grad, rtol=1e-9, atol=1e-12)
