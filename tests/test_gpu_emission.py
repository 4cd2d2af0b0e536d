"""Per-triangle emission re-estimation (Eq. 13 with f = 0) through the C ABI
against the oracle, bit for bit: segments of every size class the kernel
distinguishes (empty, one pixel, up to one wavefront, just above it, and one
triangle seen by 100,000 pixels), ties, negative values and signed zeros,
non-emitters, an output buffer full of NaN, repeated calls; and the real
pipeline on the room, whose emitters are recovered from noisy pixels."""
import numpy as np
import pytest
import torch

import synth
from oracle import emission as oe
from paper_2304_05669_amd import fipt

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _segments(rng):
    sizes = [0, 1, 2, 3, 63, 64, 65, 66, 127, 128, 129, 1000, 4097, 100000]
    T = 3000
    tri = [np.full(k, t, np.int32) for t, k in enumerate(sizes)]
    rest = rng.integers(len(sizes), T, size=150000).astype(np.int32)
    tri = np.concatenate(tri + [rest, np.full(5000, -1, np.int32)])
    rng.shuffle(tri)
    return tri, T


@pytest.mark.parametrize("kind", ["continuous", "ties"])
def test_median_bitwise_against_oracle(kind):
    rng = np.random.default_rng(11 if kind == "continuous" else 12)
    tri, T = _segments(rng)
    n = len(tri)
    if kind == "continuous":
        obs = (rng.standard_normal((3, n)) * 10).astype(np.float32)
    else:
        # few distinct values, negative ones, and both signed zeros
        obs = rng.integers(-3, 4, size=(3, n)).astype(np.float32) * 0.5
        obs[rng.uniform(size=(3, n)) < 0.1] = -0.0
    emitter = rng.uniform(size=T) < 0.6
    emitter[:14] = True                       # every size class is an emitter
    plan = fipt.EmissionPlan(tri, T)
    out = torch.full((3, T), float("nan"), dtype=torch.float32, device=DEV)
    o = torch.from_numpy(obs).to(DEV)
    e = torch.from_numpy(emitter.astype(np.uint8)).to(DEV)
    got = plan.median(o, e, out=out)
    again = plan.median(o, e)
    torch.cuda.synchronize()
    got, again = got.cpu().numpy(), again.cpu().numpy()
    want = oe.emission_median(tri, obs, T, emitter)
    np.testing.assert_array_equal(got, want)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))


def test_room_emitters_recovered():
    """The room's lamps and window, seen by its 24 cameras through noisy
    observations (emission times 1 + 0.01 z on emitter pixels, anything on
    the others): the GPU median equals the oracle's bit for bit and is
    within four standard errors of the median of the true emission for
    every emitter triangle seen by at least 9 pixels."""
    sc = synth.room()
    scene = fipt.Scene(sc.verts, sc.tris, device=0)
    try:
        planes, tri = fipt.fipt_gen_points(scene, sc.cameras)
        torch.cuda.synchronize()
        tri = tri.cpu().numpy()
    finally:
        scene.destroy()
    T = sc.n_tris
    rng = np.random.default_rng(5)
    Le = sc.emission
    emitter = Le[0] > 0
    seen = tri >= 0
    on_em = seen & emitter[np.maximum(tri, 0)]
    obs = rng.uniform(0, 1, (3, len(tri))).astype(np.float32)
    obs[:, on_em] = (Le[:, tri[on_em]] * (1 + 0.01 * rng.standard_normal((3, on_em.sum())))).astype(np.float32)
    plan = fipt.EmissionPlan(tri, T)
    got = plan.median(torch.from_numpy(obs).to(DEV), torch.from_numpy(emitter).to(DEV)).cpu().numpy()
    np.testing.assert_array_equal(got, oe.emission_median(tri, obs, T, emitter))
    counts = np.bincount(tri[seen], minlength=T)
    well_seen = emitter & (counts >= 9)
    assert well_seen.sum() > 50
    # the median of k normal samples has a standard error of ~1.2533 sigma / sqrt(k)
    tol = 4 * 1.2533 * 0.01 / np.sqrt(counts[well_seen])
    rel = np.abs(got[:, well_seen] / Le[:, well_seen] - 1)
    assert (rel <= tol).all(), rel.max()
    assert (got[:, ~emitter] == 0).all()


def test_rejects_misshapen_buffers():
    plan = fipt.EmissionPlan(np.array([0, 1, -1, 1], np.int32), 3)
    obs = torch.zeros((3, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        plan.median(obs[:, :3].contiguous(), torch.zeros(3, dtype=torch.uint8, device=DEV))
    with pytest.raises(ValueError):
        plan.median(obs, torch.zeros(4, dtype=torch.uint8, device=DEV))
    with pytest.raises(fipt.FiptError):
        fipt.EmissionPlan(np.array([0, 5], np.int32), 3)
