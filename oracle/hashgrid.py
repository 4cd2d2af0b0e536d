"""The paper's material network (Eq. 14; architecture in the supplementary
network paragraph): (a, sigma, m) = Sigmoid(MLP_brdf(hash encoding of x)),
with a multiresolution hash encoding (Mueller et al. 2022) of 32 levels and
2^19 entries per level, and an MLP of two hidden layers of 64 with ReLU.
Forward and backward in numpy float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings (the paper defers the encoding's other parameters to its
recommended defaults): 2 features per level, base resolution 16 and a
per-level scale of 2, so level l has N_l = 16 * 2^l cells per axis over the
scene box; the published spatial-hash primes (1, 2654435761, 805459861) with
32-bit wraparound, a level indexed densely when its (N_l + 1)^3 vertices fit
the table; trilinear interpolation of the cell's 8 vertices; no biases in
the MLP; outputs in the order of the material planes (a_r, a_g, a_b, sigma,
m); ReLU'(0) = 0.

The point's position in the unit cube and its cell are integer decisions
taken from floating point, so they are computed in single precision exactly
as the kernel does: p = clamp((x - lo) * inv, 0, 1) with inv = 1 / (hi - lo)
in float32, u = p N_l (exact: N_l is a power of two), cell
c = min(floor(u), N_l - 1), fraction f = u - c (exact).  Everything after
that is float64.
"""
from __future__ import annotations

import numpy as np

LEVELS = 32
FEATURES = 2
LOG2_T = 19
T = 1 << LOG2_T
BASE_RES = 16
HIDDEN = 64
OUT = 5
PRIMES = (1, 2654435761, 805459861)
N_TABLE = LEVELS * T * FEATURES
N_W1 = HIDDEN * LEVELS * FEATURES
N_W2 = HIDDEN * HIDDEN
N_W3 = OUT * HIDDEN
N_PARAMS = N_TABLE + N_W1 + N_W2 + N_W3


def split(params):
    """params [N_PARAMS] -> tables [L, T, F], W1 [64, 64], W2 [64, 64], W3 [5, 64]."""
    p = np.asarray(params, dtype=np.float64)
    o = 0
    tab = p[o:o + N_TABLE].reshape(LEVELS, T, FEATURES)
    o += N_TABLE
    W1 = p[o:o + N_W1].reshape(HIDDEN, LEVELS * FEATURES)
    o += N_W1
    W2 = p[o:o + N_W2].reshape(HIDDEN, HIDDEN)
    o += N_W2
    W3 = p[o:o + N_W3].reshape(OUT, HIDDEN)
    return tab, W1, W2, W3


def unit_position(x, lo, hi):
    """p [3, N] float32: clamp((x - lo) * inv, 0, 1), inv = 1 / (hi - lo), all
    in single precision."""
    x = np.asarray(x, dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float32)
    hi = np.asarray(hi, dtype=np.float32)
    inv = np.float32(1.0) / (hi - lo)
    p = (x - lo[:, None]) * inv[:, None]
    return np.clip(p, np.float32(0.0), np.float32(1.0)).astype(np.float32)


def level_corners(p, level: int):
    """Table indices [8, N] and trilinear weights [8, N] of the 8 vertices of
    each point's cell at one level; corner bit 0/1/2 = +1 along x/y/z."""
    n_l = np.float32(BASE_RES * 2.0 ** level)
    u = p * n_l                                    # exact in float32
    c = np.minimum(np.floor(u), n_l - np.float32(1.0))
    f = (u - c).astype(np.float64)                 # exact
    ci = c.astype(np.float64).astype(np.uint64)
    res = int(BASE_RES * 2 ** level) + 1
    dense = res ** 3 <= T
    idx = np.zeros((8, p.shape[1]), dtype=np.int64)
    w = np.ones((8, p.shape[1]))
    for k in range(8):
        xyz = []
        for a in range(3):
            bit = (k >> a) & 1
            xyz.append(ci[a] + np.uint64(bit))
            w[k] *= f[a] if bit else 1.0 - f[a]
        if dense:
            idx[k] = (xyz[0] + xyz[1] * res + xyz[2] * res * res).astype(np.int64)
        else:
            h = np.zeros(p.shape[1], dtype=np.uint64)
            for a in range(3):
                h ^= ((xyz[a] & np.uint64(0xFFFFFFFF)) * np.uint64(PRIMES[a])) & np.uint64(0xFFFFFFFF)
            idx[k] = (h & np.uint64(T - 1)).astype(np.int64)
    return idx, w


def encode(tab, p):
    """Features e [64, N]: level l's two features at rows 2l, 2l + 1."""
    N = p.shape[1]
    e = np.zeros((LEVELS * FEATURES, N))
    for l in range(LEVELS):
        idx, w = level_corners(p, l)
        for k in range(8):
            e[FEATURES * l:FEATURES * (l + 1)] += w[k] * tab[l, idx[k]].T
    return e


def forward(params, x, lo, hi):
    """Material [5, N] = Sigmoid(W3 ReLU(W2 ReLU(W1 e))) and the
    intermediates the backward pass uses."""
    tab, W1, W2, W3 = split(params)
    p = unit_position(x, lo, hi)
    e = encode(tab, p)
    z1 = W1 @ e
    h1 = np.maximum(z1, 0.0)
    z2 = W2 @ h1
    h2 = np.maximum(z2, 0.0)
    z3 = W3 @ h2
    y = 1.0 / (1.0 + np.exp(-z3))
    return y, dict(p=p, e=e, z1=z1, h1=h1, z2=z2, h2=h2, y=y)


def backward(params, x, lo, hi, grad_y):
    """Gradient of sum(grad_y * y) with respect to params (same layout)."""
    tab, W1, W2, W3 = split(params)
    _, s = forward(params, x, lo, hi)
    gy = np.asarray(grad_y, dtype=np.float64)
    d3 = gy * s["y"] * (1.0 - s["y"])
    gW3 = d3 @ s["h2"].T
    d2 = (W3.T @ d3) * (s["z2"] > 0)
    gW2 = d2 @ s["h1"].T
    d1 = (W2.T @ d2) * (s["z1"] > 0)
    gW1 = d1 @ s["e"].T
    ge = W1.T @ d1
    gtab = np.zeros_like(tab)
    for l in range(LEVELS):
        idx, w = level_corners(s["p"], l)
        for k in range(8):
            for f in range(FEATURES):
                np.add.at(gtab[l, :, f], idx[k], w[k] * ge[FEATURES * l + f])
    return np.concatenate([gtab.ravel(), gW1.ravel(), gW2.ravel(), gW3.ravel()])
