"""GPU parity of the stage-3 refinement (fipt_refine, Sec. 4.3, Eq. 10 and
11) against the oracle, through the C ABI (Python binding).

The criterion (>= 99.9 % of points within 1e-4, the rest within 1e-2 or
the oracle's envelope) is asserted where paths are well conditioned: the
whole tiny box (4096 points, 448 lobe samples each) under a smooth material
(about half of the hits glossy, paths up to eight vertices, emitter
sampling with MIS), with emitter sampling and with BRDF sampling only; a
rough random material with one glossy bounce; sampled points of the full
room (1,843,200 points, 896 samples each, the differentiation workload's
128^3 material grid, launched as the benchmark launches it) with one glossy
bounce.  Deep paths through a rough material are chaotic in any finite
precision, so at the full depth of eight vertices the rough cases are
checked by statistical agreement instead.  Also ragged counts, invalid
points, the one-vertex cap, determinism and argument checks."""
import numpy as np
import pytest
import torch

import synth
from oracle import bake as ob
from paper_2304_05669_amd import fipt
from tests.parity import (assert_bake_parity, assert_refine_parity, bake_report, max_outside,
                          stratified_points)

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
BOX = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))


def _scene(sc):
    s = fipt.Scene(sc.verts, sc.tris, device=0)
    kind = fipt.CACHE_VERTEX if sc.cache_kind == "vertex" else fipt.CACHE_TRIANGLE
    s.set_radiance(torch.from_numpy(sc.cache).to(DEV), kind, torch.from_numpy(sc.emission).to(DEV))
    return s


def smooth_grid(seed=5):
    """A 2^3 material grid over the unit box: every quantity linear between
    random corner values, roughness in [0.2, 0.9] (about half of the hits
    glossy), so a position error barely moves the next direction."""
    rng = np.random.default_rng(seed)
    g = np.empty((5, 2, 2, 2), np.float32)
    g[0:3] = rng.uniform(0.2, 0.9, size=(3, 2, 2, 2))
    g[3] = rng.uniform(0.2, 0.9, size=(2, 2, 2))
    g[4] = rng.uniform(0.0, 1.0, size=(2, 2, 2))
    return g


@pytest.fixture(scope="module")
def tiny_case():
    sc = synth.tiny_box()
    osc = ob.OracleScene(sc)
    pts, tri = ob.points_f32(ob.primary(osc))
    grid = smooth_grid()
    s = _scene(sc)
    yield sc, osc, pts, tri, grid, s
    s.destroy()


def assert_statistical_agreement(got, want, spp_d, spp_s, z_max=4.0):
    """Deep glossy paths in a rough material field are chaotic: a single-
    precision position error, coupled through the roughness gradient into
    the next direction, grows several-fold per bounce, so the GPU's and the
    oracle's paths part after a few vertices and single samples no longer
    agree.  What holds at any depth: both are the same estimator, so every
    value agrees within z_max of the oracle's standard errors (the diverged
    samples are few and bounded by them)."""
    se = ob.std_error(want, spp_d, spp_s)
    o = want["mean"]
    tau = 1e-6 * np.abs(o).max(axis=1, keepdims=True)
    z = np.abs(got - o) / np.maximum(se, tau)
    worst = float(z.max())
    assert worst < z_max, f"worst |gpu - oracle| = {worst:.2f} standard errors"
    return worst


def _refine_gpu(s, pts, tri, grid, lo, hi, spp_d, spp_s, sigma, seed, **kw):
    out = fipt.fipt_refine(s, torch.from_numpy(pts).to(DEV), torch.from_numpy(tri).to(DEV), spp_d,
                           spp_s, sigma, seed, torch.from_numpy(grid).to(DEV), lo, hi, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("flags", [0, fipt.REFINE_BSDF_ONLY])
def test_tiny_refine_parity(tiny_case, flags):
    sc, osc, pts, tri, grid, s = tiny_case
    want = ob.refine(osc, pts, tri, grid, *BOX, spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed,
                     flags=flags)
    got = _refine_gpu(s, pts, tri, grid, *BOX, sc.spp, sc.spp, sc.sigma, sc.seed, flags=flags)
    r = assert_refine_parity(got, want)
    print(f"tiny refine parity (flags {flags}):", r, "ambiguous samples", want["n_ambiguous"])
    # the refinement does change the shadings here (glossy hits are common)
    base = ob.bake(osc, pts, tri, idx=np.arange(0, sc.n_points, 16), spp_d=sc.spp, spp_s=sc.spp,
                   seed=sc.seed)["mean"]
    assert np.mean(np.abs(base - want["mean"][:, ::16]) > 1e-3 * np.abs(base).max()) > 0.2


def test_tiny_refine_parity_many_levels(tiny_case):
    """With more than 10 roughness levels (3 + 6K output slots beyond the 64
    lanes of a wavefront) the kernel takes its chunked form, 64 (lobe,
    sample) pairs per step instead of a path per lane: the same criterion
    on 1024 of the tiny box's points at K = 12."""
    sc, osc, pts, tri, grid, s = tiny_case
    sigma = np.linspace(0.05, 0.6, 12).astype(np.float32)
    idx = np.arange(0, sc.n_points, 4)
    sub, subt = np.ascontiguousarray(pts[:, idx]), np.ascontiguousarray(tri[idx])
    want = ob.refine(osc, sub, subt, grid, *BOX, spp_d=32, spp_s=32, sigma=sigma, seed=sc.seed)
    got = _refine_gpu(s, sub, subt, grid, *BOX, 32, 32, sigma, sc.seed)
    assert got.shape == (3 + 6 * 12, len(idx))
    r = assert_refine_parity(got, want)
    print("tiny refine parity, K = 12:", r)


@pytest.mark.parametrize("flags", [0, fipt.REFINE_BSDF_ONLY])
def test_tiny_rough_material_parity(tiny_case, flags):
    """A rough material (random 8^3 grid, roughness U[0.02, 1] per node):
    with one glossy bounce (emitter sampling, MIS and the continuation to a
    second vertex) the criterion holds point by point; at the full depth
    of eight vertices the results agree statistically."""
    sc, osc, pts, tri, _, s = tiny_case
    grid = synth.material_grid(8, seed=77)
    want = ob.refine(osc, pts, tri, grid, *BOX, spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed,
                     flags=flags, max_vertices=2)
    got = _refine_gpu(s, pts, tri, grid, *BOX, sc.spp, sc.spp, sc.sigma, sc.seed, flags=flags,
                      max_vertices=2)
    print(f"tiny rough refine parity, 2 vertices (flags {flags}):", assert_refine_parity(got, want))
    want = ob.refine(osc, pts, tri, grid, *BOX, spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed, flags=flags)
    got = _refine_gpu(s, pts, tri, grid, *BOX, sc.spp, sc.spp, sc.sigma, sc.seed, flags=flags)
    print(f"tiny rough refine, 8 vertices (flags {flags}): worst z",
          assert_statistical_agreement(got, want, sc.spp, sc.spp), bake_report(got, want))


def test_refine_shapes_and_degenerate_points(tiny_case):
    sc, osc, pts, tri, grid, s = tiny_case
    n = 1001                                   # ragged: not a multiple of anything
    p2 = np.ascontiguousarray(pts[:, 1000:1000 + n].copy())
    t2 = np.ascontiguousarray(tri[1000:1000 + n].copy())
    t2[3] = -1                                 # no surface
    p2[6:9, 7] = (1.0, 0.0, 0.0)               # wo in the surface plane of a floor point
    p2[3:6, 7] = (0.0, 0.0, 1.0)
    t2[7] = 0
    for spp_d, spp_s, sig, mv in ((37, 5, (0.1, 0.5, 0.9), 8), (1, 1, (0.3,), 16),
                                  (20, 9, tuple(np.linspace(0.05, 1.0, 12)), 3)):
        want = ob.refine(osc, p2, t2, grid, *BOX, spp_d=spp_d, spp_s=spp_s, sigma=sig, seed=4,
                         max_vertices=mv)
        got = _refine_gpu(s, p2, t2, grid, *BOX, spp_d, spp_s, sig, 4, max_vertices=mv)
        assert np.all(got[:, 3] == 0.0) and np.all(got[:, 7] == 0.0)
        assert_refine_parity(got, want)


def test_one_vertex_cap_matches_the_bake(tiny_case):
    """With paths capped at one vertex the refinement is the stage-1 bake
    (for a cache that is zero on the emitters): against the oracle's bake."""
    sc0, _, pts, tri, grid, _ = tiny_case
    sc = synth.tiny_box()
    sc.cache[:, sc.emission.max(axis=0) > 0] = 0.0
    osc = ob.OracleScene(sc)
    s = _scene(sc)
    idx = np.arange(0, sc.n_points, 3)
    want = ob.bake(osc, pts, tri, idx=idx, spp_d=32, spp_s=16, seed=8)
    got = _refine_gpu(s, pts, tri, grid, *BOX, 32, 16, sc.sigma, 8, max_vertices=1)[:, idx]
    assert_bake_parity(got, want, min_frac=1.0 - max_outside(len(idx)) / len(idx))
    s.destroy()


def test_refine_is_deterministic(tiny_case):
    sc, osc, pts, tri, grid, s = tiny_case
    a = _refine_gpu(s, pts, tri, grid, *BOX, 16, 16, sc.sigma, 3)
    b = _refine_gpu(s, pts, tri, grid, *BOX, 16, 16, sc.sigma, 3)
    np.testing.assert_array_equal(a, b)


def test_refine_arguments_rejected(tiny_case):
    sc, osc, pts, tri, grid, s = tiny_case
    P, T = torch.from_numpy(pts).to(DEV), torch.from_numpy(tri).to(DEV)
    G = torch.from_numpy(grid).to(DEV)
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(s, P, T, 4, 4, sc.sigma, 1, G, *BOX, max_vertices=0)
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(s, P, T, 4, 4, sc.sigma, 1, G, *BOX, max_vertices=17)
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(s, P, T, 4, 4, sc.sigma, 1, G, BOX[1], BOX[0])
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(s, P, T, 4, 4, sc.sigma, 1, G, *BOX, flags=2)
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(s, P, T, 0, 4, sc.sigma, 1, G, *BOX)
    # a scene with a voxel cache is refused
    sv = fipt.Scene(sc.verts, sc.tris, device=0)
    sv.set_voxel_radiance(torch.zeros((3, 8 ** 3), device=DEV), 8, *BOX)
    with pytest.raises(fipt.FiptError):
        fipt.fipt_refine(sv, P, T, 4, 4, sc.sigma, 1, G, *BOX)
    sv.destroy()


def _room_refine_case(grid, n_sample, max_vertices, seed=51, chunk=32, perturbations=0):
    """Full-size refinement of the room (1,843,200 points, 896 samples each),
    launched as the benchmark launches it; the oracle on stratified points
    baking the same inputs (its own shading points written into the GPU
    buffer).  With `perturbations`, the oracle also bakes that many copies of
    the sampled points with each normal turned by a random 1e-7 rad (the
    size of a single-precision direction's rounding), and the largest change
    they cause is returned per value."""
    import sys
    import time
    sc = synth.room()
    s = _scene(sc)
    planes, tri_g = fipt.fipt_gen_points(s, sc.cameras)
    torch.cuda.synchronize()
    idx = stratified_points(sc.n_points, n_sample, seed)
    osc = ob.OracleScene(sc)
    p32, t32 = ob.points_f32(ob.primary(osc, idx=idx))
    ii = torch.from_numpy(idx).to(DEV)
    planes[:, ii] = torch.from_numpy(p32).to(DEV)
    tri_g[ii] = torch.from_numpy(t32).to(DEV)
    out = fipt.fipt_refine(s, planes, tri_g, sc.spp, sc.spp, sc.sigma, sc.seed,
                           torch.from_numpy(grid).to(DEV), sc.bmin, sc.bmax,
                           max_vertices=max_vertices)
    torch.cuda.synchronize()
    got = out[:, ii].cpu().numpy()
    s.destroy()
    t0 = time.perf_counter()

    def oracle(P, label):
        full_p = np.zeros((9, sc.n_points), np.float32)
        full_t = np.full(sc.n_points, -1, np.int32)
        full_p[:, idx] = P
        full_t[idx] = t32
        parts = []
        for a in range(0, len(idx), chunk):
            parts.append(ob.refine(osc, full_p, full_t, grid, sc.bmin, sc.bmax, idx=idx[a:a + chunk],
                                   spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed,
                                   max_vertices=max_vertices))
            print(f"oracle room refine ({label}): {min(a + chunk, len(idx))}/{len(idx)} points "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
        return {k: np.concatenate([p[k] for p in parts], axis=1) for k in ("mean", "lo", "hi", "sq")}

    want = oracle(p32, "nominal")
    moved = np.zeros_like(want["mean"])
    rng = np.random.default_rng(seed)
    for k in range(perturbations):
        P = p32.astype(np.float64)
        nrm = P[3:6] + rng.normal(size=P[3:6].shape) * 1e-7
        P[3:6] = nrm / np.linalg.norm(nrm, axis=0)
        moved = np.maximum(moved, np.abs(oracle(P.astype(np.float32), f"perturbed {k + 1}")["mean"]
                                          - want["mean"]))
    return sc, got, want, moved


def test_room_refine_smooth_material_parity():
    """A smooth material over the room (2^3 grid, roughness 0.2-0.9: about
    half of the hits glossy) at the full depth of eight vertices: the
    criterion point by point on 128 stratified points."""
    g = smooth_grid(seed=9)
    sc, got, want, _ = _room_refine_case(g, 128, 8, seed=52)
    print("room refine, smooth material, 8 vertices:", assert_refine_parity(got, want))


def test_room_refine_rough_material_parity():
    """The differentiation workload's 128^3 material grid (roughness
    U[0.02, 1] per node, 4.7 cm apart) with one glossy bounce.  There a
    position error at the glossy hit, through the roughness gradient, turns
    the next direction: turning the input normals by 1e-7 rad moves about a
    third of the oracle's own points by more than 1e-4.  The tolerance per
    value is the larger of 1e-4 and four times the change two such
    perturbations cause in the oracle; the criterion is otherwise the
    bake's."""
    grid = synth.material_grid(128, seed=1006)
    sc, got, want, moved = _room_refine_case(grid, 128, 2, perturbations=2)
    o = want["mean"]
    tau = 1e-6 * np.abs(o).max(axis=1, keepdims=True)
    tol = np.maximum(1e-4, 4.0 * moved / np.maximum(np.abs(o), tau))
    print("room refine, rough material, 2 vertices:", assert_refine_parity(got, want, tol),
          "largest tolerance", float(tol.max()))


def test_room_refine_benchmark_setting_agrees():
    """The benchmark's setting (the 128^3 rough material, eight vertices):
    deep glossy paths there are chaotic, so statistical agreement on 48
    stratified points."""
    grid = synth.material_grid(128, seed=1006)
    sc, got, want, _ = _room_refine_case(grid, 48, 8, seed=53, chunk=16)
    print("room refine, rough material, 8 vertices: worst z",
          assert_statistical_agreement(got, want, sc.spp, sc.spp), bake_report(got, want))
