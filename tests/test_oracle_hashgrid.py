"""Pins of the oracle's hash-grid material network (Eq. 14):

* vertex indices by hand: a dense level (row-major over its (N + 1)^3
  vertices) and a hashed level (the three primes, 32-bit wraparound,
  computed here with Python integers), and the far face p = 1 clamped into
  the last cell with weight 1 on its upper vertex;
* trilinear weights are non-negative and sum to one; on the dense levels a
  table holding an affine function of the vertex coordinates is
  interpolated exactly;
* zero weights give outputs of exactly 1/2;
* the backward pass against central finite differences in float64 on table
  entries and weights of every layer, and against torch float64 autograd of
  an independently written forward pass (gather + sum per level).
"""
import numpy as np
import pytest
import torch

from oracle import hashgrid as hg

LO = np.array([-1.0, 0.0, 2.0], np.float32)
HI = np.array([3.0, 2.0, 3.0], np.float32)


def _params(seed, scale_tab=0.1):
    rng = np.random.default_rng(seed)
    p = np.zeros(hg.N_PARAMS)
    p[:hg.N_TABLE] = rng.uniform(-scale_tab, scale_tab, hg.N_TABLE)
    p[hg.N_TABLE:] = rng.standard_normal(hg.N_PARAMS - hg.N_TABLE) / 8.0
    return p


def _points(n, seed):
    rng = np.random.default_rng(seed)
    return (LO[:, None] + rng.uniform(0, 1, (3, n)) * (HI - LO)[:, None]).astype(np.float32)


def test_indices_by_hand():
    p = np.array([[0.5], [0.25], [0.0]], np.float32)
    idx, w = hg.level_corners(p, 0)                 # N = 16, 17^3 vertices, dense
    assert idx[0, 0] == 8 + 4 * 17 and w[0, 0] == 1.0 and np.all(w[1:, 0] == 0.0)
    # corner 7 = (+1, +1, +1)
    assert idx[7, 0] == 9 + 5 * 17 + 1 * 17 * 17
    p = np.array([[0.5], [0.5], [0.5]], np.float32)
    idx, w = hg.level_corners(p, 3)                 # N = 128, hashed
    m = 0xFFFFFFFF
    want = ((64 * 1) & m) ^ ((64 * 2654435761) & m) ^ ((64 * 805459861) & m)
    assert idx[0, 0] == want & (hg.T - 1)
    want7 = ((65 * 1) & m) ^ ((65 * 2654435761) & m) ^ ((65 * 805459861) & m)
    assert idx[7, 0] == want7 & (hg.T - 1)
    # the far face: last cell, all weight on the upper vertex
    p = np.array([[1.0], [1.0], [1.0]], np.float32)
    idx, w = hg.level_corners(p, 1)                 # N = 32, 33^3, dense
    assert idx[7, 0] == 32 + 32 * 33 + 32 * 33 * 33 and w[7, 0] == 1.0


def test_weights_partition_unity():
    p = hg.unit_position(_points(500, 1), LO, HI)
    for l in (0, 5, 17, 31):
        _, w = hg.level_corners(p, l)
        assert np.all(w >= 0)
        np.testing.assert_allclose(w.sum(axis=0), 1.0, rtol=1e-14)


def test_affine_table_interpolated_exactly():
    p = hg.unit_position(_points(300, 2), LO, HI)
    tab = np.zeros((hg.LEVELS, hg.T, hg.FEATURES))
    for l in range(3):                              # the dense levels
        res = hg.BASE_RES * 2 ** l + 1
        v = np.arange(res ** 3)
        x, y, z = v % res, (v // res) % res, v // (res * res)
        tab[l, :res ** 3, 0] = 0.5 * x - 0.25 * y + 2.0 * z
        tab[l, :res ** 3, 1] = 1.0 + x
    e = hg.encode(tab, p)
    for l in range(3):
        u = p.astype(np.float64) * (hg.BASE_RES * 2 ** l)
        np.testing.assert_allclose(e[2 * l], 0.5 * u[0] - 0.25 * u[1] + 2.0 * u[2], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(e[2 * l + 1], 1.0 + u[0], rtol=1e-12)


def test_zero_weights_give_one_half():
    params = _params(3)
    params[hg.N_TABLE:] = 0.0
    y, _ = hg.forward(params, _points(50, 4), LO, HI)
    assert np.all(y == 0.5)


def test_backward_finite_differences():
    params = _params(5)
    x = _points(40, 6)
    gy = np.random.default_rng(7).standard_normal((5, 40))
    g = hg.backward(params, x, LO, HI, gy)
    # probe table entries that the points touch, and weights of each layer
    s = hg.forward(params, x, LO, HI)[1]
    probes = []
    for l in (0, 4, 20, 31):
        idx, _ = hg.level_corners(s["p"], l)
        probes.append(l * hg.T * hg.FEATURES + int(idx[3, 7]) * hg.FEATURES + 1)
    probes += [hg.N_TABLE + 5, hg.N_TABLE + hg.N_W1 + 100, hg.N_TABLE + hg.N_W1 + hg.N_W2 + 7]
    eps = 1e-6
    for k in probes:
        pp, pm = params.copy(), params.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (np.sum(gy * hg.forward(pp, x, LO, HI)[0]) - np.sum(gy * hg.forward(pm, x, LO, HI)[0])) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_matches_torch_autograd():
    params = _params(8)
    x = _points(60, 9)
    gy = np.random.default_rng(10).standard_normal((5, 60))
    y, s = hg.forward(params, x, LO, HI)
    g = hg.backward(params, x, LO, HI, gy)
    P = torch.tensor(params, requires_grad=True)
    tab = P[:hg.N_TABLE].reshape(hg.LEVELS, hg.T, hg.FEATURES)
    o = hg.N_TABLE
    W1 = P[o:o + hg.N_W1].reshape(64, 64)
    W2 = P[o + hg.N_W1:o + hg.N_W1 + hg.N_W2].reshape(64, 64)
    W3 = P[o + hg.N_W1 + hg.N_W2:].reshape(5, 64)
    feats = []
    for l in range(hg.LEVELS):
        idx, w = hg.level_corners(s["p"], l)
        I = torch.tensor(idx)
        Wt = torch.tensor(w)
        f = (tab[l][I] * Wt[..., None]).sum(0)      # [N, F]
        feats.append(f.T)
    e = torch.cat(feats, 0)
    out = torch.sigmoid(W3 @ torch.relu(W2 @ torch.relu(W1 @ e)))
    (out * torch.tensor(gy)).sum().backward()
    np.testing.assert_allclose(out.detach().numpy(), y, rtol=1e-13)
    np.testing.assert_allclose(P.grad.numpy(), g, rtol=1e-10, atol=1e-14)
