"""Per-triangle emission re-estimation (Sec. 4.4, Eq. 13), in numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Under the paper's assumption that an emitter reflects no light (f = 0),
the argmin of Eq. 13 for a triangle classified as an emitter is, per colour
channel, the median of the observed values of all input pixels whose
primary hit is that triangle.  Readings where the paper is silent: the
median is taken per channel; for an even number of pixels it is the lower
of the two middle values (an element of the data, so the GPU result can be
compared bit for bit); a triangle that is not an emitter, or that no pixel
sees, gets zero emission.
"""
from __future__ import annotations

import numpy as np


def emission_median(tri, observed, n_tris: int, emitter):
    """tri [n] int (primary-hit triangle per pixel, -1 for none),
    observed [3, n] float32, emitter [n_tris] bool -> Le [3, n_tris] float32."""
    tri = np.asarray(tri, dtype=np.int64)
    obs = np.asarray(observed, dtype=np.float32)
    emitter = np.asarray(emitter, dtype=bool)
    out = np.zeros((3, n_tris), dtype=np.float32)
    for t in np.flatnonzero(emitter):
        pix = np.flatnonzero(tri == t)
        k = len(pix)
        if k == 0:
            continue
        for c in range(3):
            vals = np.sort(obs[c, pix], kind="stable")
            out[c, t] = vals[(k - 1) // 2]
    return out
