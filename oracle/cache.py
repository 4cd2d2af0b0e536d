"""The radiance cache L' as the paper builds it (Sec. 4.2, the query of
Eq. 9): every observed pixel is average-pooled into the voxel of a grid over
the scene that contains its surface point, and a query returns the value of
the voxel that contains the query point (nearest voxel).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Voxel (i, j, k) of an R^3 grid over the box [lo, hi] holds the points whose
coordinates give floor((x - lo) R / (hi - lo)) = (i, j, k) axis by axis,
clamped to [0, R - 1] (points outside the box fall into the border voxels);
its linear index is (k R + j) R + i.  Readings where the paper is silent:
the grid spans the given box (the scene's bounds), an empty voxel holds
zero, and the average is the plain mean of the pooled pixels per channel.
"""
from __future__ import annotations

import numpy as np


def voxel_of(x, lo, hi, res: int) -> np.ndarray:
    """Linear voxel index of points x [3, N] (double arithmetic on the
    float32 inputs promoted exactly)."""
    x = np.asarray(x, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ijk = []
    for a in range(3):
        u = (x[a] - lo[a]) * res / (hi[a] - lo[a])
        ijk.append(np.clip(np.floor(u), 0, res - 1).astype(np.int64))
    return (ijk[2] * res + ijk[1]) * res + ijk[0]


def voxel_pool(x, observed, lo, hi, res: int):
    """Average pooling of observed radiance [3, N] at points x [3, N] onto an
    R^3 grid.  Returns (cache [3, R^3] float64, counts [R^3] int64); the sum
    of a voxel runs over its points in index order."""
    v = voxel_of(x, lo, hi, res)
    obs = np.asarray(observed, dtype=np.float64)
    nv = res ** 3
    counts = np.bincount(v, minlength=nv).astype(np.int64)
    sums = np.zeros((3, nv))
    for c in range(3):
        np.add.at(sums[c], v, obs[c])
    cache = np.zeros((3, nv))
    seen = counts > 0
    cache[:, seen] = sums[:, seen] / counts[seen]
    return cache, counts
