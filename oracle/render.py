"""Factored re-render, photometric loss and its gradient, and the trilinear
material grid with its adjoint, in numpy float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definitions followed (Factorized Inverse Path Tracing, Sec. 3-4):
* Eq. 5: Lr = kd * Ld + ks * Ls0(sigma) + Ls1(sigma), per colour channel;
* notation table / Eq. 1: kd = a (1 - m), ks = 0.04 (1 - m) + a m;
* Eq. 8: Ls0, Ls1 at roughness sigma are linear interpolations between the
  two tabulated levels that bracket sigma;
* Eq. 2 / Eq. 15: l = sum over pixels and channels of
  (Gamma(Lr) - Gamma(Lgt))^2, Gamma the identity unless a tone map is
  asked for.

* Sec. 4.4, Eq. 12 / Eq. 15: with an emission mask alpha per point the
  rendered value compared with Lgt is (1 - alpha) Lr + alpha Lgt;
* Sec. 4.5, Eq. 17: the diffuse prior
  l_d = lambda_d * sum over points of (|1 - sigma| + |m|).

Readings where the paper is silent: below the first level or above the last
the interpolation clamps (zero roughness gradient); at an interior knot the
right-hand segment is used; the optional tone map is
Gamma(x) = sRGB-OETF(log(1 + max(x, 0))).  The prior's derivative takes
sign(0) = 0 at the kinks of the absolute values (sigma = 1, m = 0), and its
roughness term is not clamped by the interpolation bracket.
"""
from __future__ import annotations

import numpy as np


def bracket(sigma_grid, s):
    """Segment index j (largest j with sigma_j <= s, clamped to [0, K-2]),
    interpolation weight t in [0, 1] and a flag marking clamped points."""
    g = np.asarray(sigma_grid, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    K = len(g)
    j = np.searchsorted(g, s, side="right") - 1
    j = np.clip(j, 0, K - 2)
    t = (s - g[j]) / (g[j + 1] - g[j])
    clamped = (s < g[0]) | (s > g[-1])
    t = np.clip(t, 0.0, 1.0)
    return j, t, clamped


def _srgb(x):
    return np.where(x <= 0.0031308, 12.92 * x, 1.055 * np.power(np.maximum(x, 0.0031308), 1.0 / 2.4) - 0.055)


def _srgb_d(x):
    return np.where(x <= 0.0031308, 12.92,
                    1.055 / 2.4 * np.power(np.maximum(x, 0.0031308), 1.0 / 2.4 - 1.0))


def tonemap(x, kind: int):
    x = np.asarray(x, dtype=np.float64)
    if kind == 0:
        return x
    y = np.log1p(np.maximum(x, 0.0))
    return _srgb(y)


def tonemap_d(x, kind: int):
    x = np.asarray(x, dtype=np.float64)
    if kind == 0:
        return np.ones_like(x)
    xp = np.maximum(x, 0.0)
    y = np.log1p(xp)
    return np.where(x > 0.0, _srgb_d(y) / (1.0 + xp), 0.0)


def _levels(shading, K):
    sh = np.asarray(shading, dtype=np.float64)
    N = sh.shape[1]
    Ld = sh[0:3]
    Ls0 = sh[3:3 + 3 * K].reshape(K, 3, N)
    Ls1 = sh[3 + 3 * K:3 + 6 * K].reshape(K, 3, N)
    return Ld, Ls0, Ls1


def render(shading, material, sigma_grid):
    """Lr [3, N] plus the intermediates the gradient needs."""
    K = len(sigma_grid)
    Ld, Ls0, Ls1 = _levels(shading, K)
    mat = np.asarray(material, dtype=np.float64)
    a, s, m = mat[0:3], mat[3], mat[4]
    N = mat.shape[1]
    j, t, clamped = bracket(sigma_grid, s)
    cols = np.arange(N)
    S0j, S0k = Ls0[j, :, cols].T, Ls0[j + 1, :, cols].T     # [3, N]
    S1j, S1k = Ls1[j, :, cols].T, Ls1[j + 1, :, cols].T
    L0 = (1.0 - t) * S0j + t * S0k
    L1 = (1.0 - t) * S1j + t * S1k
    kd = a * (1.0 - m)
    ks = 0.04 * (1.0 - m) + a * m
    Lr = kd * Ld + ks * L0 + L1
    g = np.asarray(sigma_grid, dtype=np.float64)
    dsig = g[j + 1] - g[j]
    return dict(Lr=Lr, L0=L0, L1=L1, Ld=Ld, a=a, m=m, ks=ks, dS0=S0k - S0j,
                dS1=S1k - S1j, dsig=dsig, clamped=clamped)


def loss_and_grad(shading, material, observed, sigma_grid, tone: int = 0):
    """Sum-of-squares loss and its gradient with respect to the per-point
    material [5, N] (a_r, a_g, a_b, roughness, metallic)."""
    r = render(shading, material, sigma_grid)
    Lgt = np.asarray(observed, dtype=np.float64)
    res = tonemap(r["Lr"], tone) - tonemap(Lgt, tone)
    loss = float(np.sum(res * res))
    g = 2.0 * res * tonemap_d(r["Lr"], tone)                     # dl/dLr [3, N]
    grad = np.zeros((5, g.shape[1]))
    grad[0:3] = g * ((1.0 - r["m"]) * r["Ld"] + r["m"] * r["L0"])
    grad[4] = np.sum(g * (-r["a"] * r["Ld"] + (r["a"] - 0.04) * r["L0"]), axis=0)
    dsig = np.sum(g * (r["ks"] * r["dS0"] + r["dS1"]), axis=0) / r["dsig"]
    grad[3] = np.where(r["clamped"], 0.0, dsig)
    return loss, grad, r["Lr"]


def masked_loss_and_grad(shading, material, observed, alpha, sigma_grid, tone: int = 0,
                         lambda_d: float = 0.0):
    """Emission-masked photometric loss (Eq. 12 / 15) plus the diffuse prior
    (Eq. 17), with its gradients.

    alpha [N] is the emission mask; the loss is
      sum over points and channels of (Gamma((1 - alpha) Lr + alpha Lgt) - Gamma(Lgt))^2
      + lambda_d * sum over points of (|1 - sigma| + |m|).
    Returns (loss, grad [5, N] with respect to the material, grad_alpha [N],
    Lr [3, N]); Lr is the unmasked reflected radiance."""
    r = render(shading, material, sigma_grid)
    Lgt = np.asarray(observed, dtype=np.float64)
    al = np.asarray(alpha, dtype=np.float64)[None, :]
    Lr = r["Lr"]
    Lhat = (1.0 - al) * Lr + al * Lgt
    res = tonemap(Lhat, tone) - tonemap(Lgt, tone)
    mat = np.asarray(material, dtype=np.float64)
    sig, met = mat[3], mat[4]
    prior = lambda_d * np.sum(np.abs(1.0 - sig) + np.abs(met))
    loss = float(np.sum(res * res) + prior)
    gh = 2.0 * res * tonemap_d(Lhat, tone)                       # dl/dLhat [3, N]
    g = gh * (1.0 - al)                                          # dl/dLr
    grad = np.zeros((5, g.shape[1]))
    grad[0:3] = g * ((1.0 - r["m"]) * r["Ld"] + r["m"] * r["L0"])
    grad[4] = np.sum(g * (-r["a"] * r["Ld"] + (r["a"] - 0.04) * r["L0"]), axis=0)
    dsig = np.sum(g * (r["ks"] * r["dS0"] + r["dS1"]), axis=0) / r["dsig"]
    grad[3] = np.where(r["clamped"], 0.0, dsig)
    grad[3] += -lambda_d * np.sign(1.0 - sig)
    grad[4] += lambda_d * np.sign(met)
    grad_alpha = np.sum(gh * (Lgt - Lr), axis=0)
    return loss, grad, grad_alpha, Lr


# -------------------------------------------------------------------------
# trilinear material grid (vertex-aligned over the box [bmin, bmax])
# -------------------------------------------------------------------------
def _cell(x, bmin, bmax, res):
    x = np.asarray(x, dtype=np.float64)
    bmin = np.asarray(bmin, dtype=np.float64)[:, None]
    bmax = np.asarray(bmax, dtype=np.float64)[:, None]
    u = (x - bmin) / (bmax - bmin) * (res - 1)
    u = np.clip(u, 0.0, res - 1)
    i0 = np.minimum(np.floor(u).astype(np.int64), res - 2)
    f = u - i0
    return i0, f


def grid_gather(grid, x, bmin, bmax):
    """grid [C, R, R, R] (x fastest), points x [3, N] -> values [C, N].
    Node (i, j, k) sits at bmin + (i, j, k) * (bmax - bmin) / (R - 1);
    coordinates outside the box are clamped onto it."""
    g = np.asarray(grid, dtype=np.float64)
    C, R = g.shape[0], g.shape[1]
    i0, f = _cell(x, bmin, bmax, R)
    out = np.zeros((C, i0.shape[1]))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1])
                     * (f[2] if dz else 1 - f[2]))
                out += w * g[:, i0[2] + dz, i0[1] + dy, i0[0] + dx]
    return out


def grid_scatter(grad_points, x, bmin, bmax, res):
    """Adjoint of grid_gather: sum of each point's gradient into the eight
    nodes of its cell with the same trilinear weights."""
    gp = np.asarray(grad_points, dtype=np.float64)
    C = gp.shape[0]
    i0, f = _cell(x, bmin, bmax, res)
    out = np.zeros((C, res, res, res))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1])
                     * (f[2] if dz else 1 - f[2]))
                for c in range(C):
                    np.add.at(out[c], (i0[2] + dz, i0[1] + dy, i0[0] + dx), w * gp[c])
    return out
