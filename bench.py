"""Benchmark of the factorized-shading hot path on one MI355X.

One step = the whole hot path over the synthetic room (189,440 triangles,
24 cameras x 320 x 240 = 1,843,200 shading points, 128 samples per lobe,
6 roughness levels):
  shading points from the cameras -> bake of Ld, Ls0[6], Ls1[6]
  (1,651,507,200 lobe samples) -> material gather from a 128^3 grid ->
  factored re-render + loss + gradient -> gradient scatter to the grid.

Prints one JSON line.  `value` is lobe samples baked per second over whole
steps (inputs resident in HBM).  Per-kernel times come from HIP events on
the stream the kernels run on.  The serving leg replays a Poisson trace of
bake requests against the continuous-batching server and against
one-request-at-a-time baking and reports p50/p99 latency.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_2304_05669_amd import fipt  # noqa: E402

PEAK_HBM_GBS = 8000.0
# published vector FP32 peak of MI355X (256 CUs at 2.4 GHz, packed FMA)
PEAK_FP32_TFLOPS = 157.3
# algorithmic flops per unit of bake work, counted as the hot path's scope
# counts them: ~20 per ray-box slab test (four per 4-wide node visited), ~30
# per ray-triangle test, ~100 per lobe sample (random numbers, direction,
# weights)
FLOPS_PER_NODE = 4 * 20
FLOPS_PER_CHAIN_LEVEL = 3 * 20   # a chain level tests the three siblings
FLOPS_PER_TRI = 30
FLOPS_PER_SAMPLE = 100
# Secondary figure: the VALU issue rate of MI355X, 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz, one operation per lane per cycle (packed FP32
# instructions are not used), against operations counted per instruction
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic VALU operations per unit of bake work
OPS_PER_NODE = 81      # 4-wide node: four slab tests (6 FMA, 12 min/max, 1 compare
                       # each) and a five-comparator ordering of the hit children
OPS_PER_CHAIN_LEVEL = 60   # three slab tests of siblings below a point's chain, three comparators
OPS_PER_TRI = 40       # Moller-Trumbore: 2 cross products, 4 dots, reciprocal, compares
OPS_PER_SAMPLE = 180   # Philox4x32-10 (~100 integer ops) + direction and weights
OPS_PER_HIT = 12       # radiance: barycentric blend of the corner cache + emission
# render-loss bytes per point: material 20 + Ld 12 + two bracketing levels
# of Ls0/Ls1 48 + Lgt 12 + gradient 20
LOSS_BYTES_PER_POINT = 112
# the masked loss also reads alpha and writes d loss / d alpha
MASKED_LOSS_BYTES_PER_POINT = 120
# fused material fetch + loss + adjoint, per point: position 12 B, Ld 12 B,
# the bracketing levels of Ls0 and Ls1 48 B, Lgt 12 B (material and its
# gradient stay on chip or in the grid, counted once per grid)
FUSED_LOSS_BYTES_PER_POINT = 84
LAMBDA_D = 5e-4        # weight of the diffuse prior, as in Eq. 17
VOXEL_RES = 256        # the radiance cache grid of Sec. 4.2
# hash-grid network forward, per point: 8 B per table vertex read (those of
# non-zero weight, counted per run), 12 B position in, 20 B material out;
# 2 (64*64 + 64*64 + 5*64) multiply-adds as flops
HG_FWD_FLOPS_PER_POINT = 2 * (64 * 64 + 64 * 64 + 5 * 64)
SHADING_PLANES = 39
COUNTERS = os.path.join(ROOT, "profiles", "counters_room.json")
# the sources each measured kernel is built from
KERNEL_SOURCES = {
    "k_bake": ("bake.hip", "device.hpp", "fipt_internal.hpp", "bvh_build.cpp"),
    "k_render_loss": ("loss.hip", "fipt_internal.hpp"),
    "k_render_loss_masked": ("loss.hip", "fipt_internal.hpp"),
    "k_bake_voxel": ("bake.hip", "device.hpp", "fipt_internal.hpp", "bvh_build.cpp"),
    "k_hg_forward": ("hashgrid.hip", "fipt_internal.hpp"),
    "k_hg_forward_save": ("hashgrid.hip", "fipt_internal.hpp"),
    "k_hg_backward": ("hashgrid.hip", "fipt_internal.hpp"),
    "k_hg_table_grad": ("hashgrid.hip", "fipt_internal.hpp"),
    "k_grid_adjoint": ("loss.hip", "grid.cpp", "fipt_internal.hpp"),
    "k_grid_gather": ("loss.hip", "fipt_internal.hpp"),
    "k_grid_render_loss": ("loss.hip", "grid.cpp", "fipt_internal.hpp"),
}


def sources_sha(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2304_05669_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, for each
    kernel whose sources are unchanged since the counters were taken."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return {}
    out = {}
    for k, v in c.get("kernels", {}).items():
        if k in KERNEL_SOURCES and v.get("sources_sha") == sources_sha(k):
            out[k] = v.get("hbm_bytes_per_launch")
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Timer:
    """HIP events on torch's current stream (where the library launches)."""

    def __init__(self):
        self.ev = {}

    def mark(self, name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        self.ev.setdefault(name, []).append(e)

    def spans(self, a, b):
        return [x.elapsed_time(y) for x, y in zip(self.ev[a], self.ev[b])]


def setup_room(sc, dev):
    scene = fipt.Scene(sc.verts, sc.tris, device=0)
    kind = fipt.CACHE_VERTEX if sc.cache_kind == "vertex" else fipt.CACHE_TRIANGLE
    scene.set_radiance(torch.from_numpy(sc.cache).to(dev), kind,
                       torch.from_numpy(sc.emission).to(dev))
    return scene


def traversal_bytes(scene, planes, tri, sc, out):
    """Algorithmic bytes of one bake launch, from the instrumented kernel:
    80 B per 4-wide BVH node visited (the half-precision planes, origin and
    child references the node step reads of its 128-byte line), 48 B per
    triangle tested, 48 B radiance record per hit, 40 B per point read and
    156 B per point written."""
    stats = torch.zeros(7, dtype=torch.int64, device=planes.device)
    fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=out, stats=stats)
    torch.cuda.synchronize()
    rays, nodes, tris, hits, node_steps, tri_steps, chain = [int(v) for v in stats.cpu()]
    n = planes.shape[1]
    P = 3 + 6 * len(sc.sigma)
    samples = n * sc.spp * (1 + len(sc.sigma))
    # a chain level's node is read once per wavefront (scalar loads), not
    # per lane: its bytes are not counted per ray
    total = nodes * 80 + tris * 48 + hits * 48 + n * 40 + n * P * 4
    ops = (nodes * OPS_PER_NODE + chain * OPS_PER_CHAIN_LEVEL + tris * OPS_PER_TRI +
           samples * OPS_PER_SAMPLE + hits * OPS_PER_HIT)
    flops = (nodes * FLOPS_PER_NODE + chain * FLOPS_PER_CHAIN_LEVEL + tris * FLOPS_PER_TRI +
             samples * FLOPS_PER_SAMPLE)
    return dict(rays=rays, nodes=nodes, tris=tris, hits=hits, samples=samples, bytes=total,
                ops=ops, flops=flops, chain_levels=chain,
                chain_levels_per_ray=chain / max(rays, 1),
                nodes_per_ray=nodes / max(rays, 1), tris_per_ray=tris / max(rays, 1),
                node_loop_lane_use=nodes / max(64 * node_steps, 1),
                tri_loop_lane_use=tris / max(64 * tri_steps, 1))


def oracle_bake_rate(sc, budget_s, seed):
    """The bake oracle (double precision, every ray against every triangle)
    on a bounded random sample of a workload's points, with every host
    thread; its shading points are the oracle's own (camera rays cast by the
    oracle).  Returns points, seconds, Gsamples/s, threads."""
    from oracle import bake as ob
    osc = ob.OracleScene(sc)
    threads = ob.max_threads()
    S = sc.spp * (1 + len(sc.sigma))
    rng = np.random.default_rng(seed)

    def run(k):
        idx = np.sort(rng.choice(sc.n_points, k, replace=False)).astype(np.int64)
        p32, t32 = ob.points_f32(ob.primary(osc, idx=idx))
        t0 = time.perf_counter()
        ob.bake(osc, p32, t32, spp_d=sc.spp, spp_s=sc.spp, seed=sc.seed, threads=threads)
        return k, time.perf_counter() - t0

    # calibrate on one point per thread, then size the sample to the budget
    # (the calibration run stands if it already took half the budget)
    k, dt = run(threads)
    if dt < 0.5 * budget_s:
        k, dt = run(min(sc.n_points, max(1, int(budget_s / max(dt, 1e-3))) * threads))
    g = k * S / dt / 1e9
    return dict(points=k, seconds=dt, gsamples_per_s=g, threads=threads,
                per_core_gsamples_per_s=g / threads,
                full_workload_extrapolated_s=sc.n_points * S / (g * 1e9))


def cpu_baseline(sc, budget_s, large_sc=None, large_budget_s=0.0, loss=None):
    """The oracle timed on the host cores: the bake oracle on a bounded
    sample of the room (the headline figure), on a smaller sample of the
    2M-triangle room, and the loss+gradient oracle (numpy float64) over a
    full room-sized point set."""
    r = oracle_bake_rate(sc, budget_s, 0)
    S = sc.spp * (1 + len(sc.sigma))
    out = dict(value=r["gsamples_per_s"], unit="Gsamples/s", cores=r["threads"], kind="oracle",
               sample=f"{r['points']} random points of the room x {S} lobe samples, brute-force "
                      f"float64 over all {sc.n_tris} triangles, {r['seconds']:.1f} s",
               per_core_gsamples_per_s=r["per_core_gsamples_per_s"],
               room_full_bake_extrapolated_s=r["full_workload_extrapolated_s"])
    if large_sc is not None and large_budget_s > 0:
        lr = oracle_bake_rate(large_sc, large_budget_s, 1)
        out["large_room"] = dict(lr, sample=f"{lr['points']} random points of the "
                                             f"{large_sc.n_tris:,}-triangle room x "
                                             f"{large_sc.spp * (1 + len(large_sc.sigma))} lobe samples")
    if loss is not None:
        out["loss_grad"] = loss
    return out


# Synthetic inputs of the loss+gradient oracle (a room-sized point set) and
# the worker pool that times it on all cores.  Both are made before anything
# initialises the GPU, so the workers are forked from a process without GPU
# state; they inherit the inputs and return their chunk's loss and gradient.
_LOSS_IN = None


def _loss_chunk(bounds):
    from oracle import render as orr
    a, b = bounds
    sh, mat, obs, sig = _LOSS_IN
    loss, grad, _ = orr.loss_and_grad(sh[:, a:b], mat[:, a:b], obs[:, a:b], sig)
    return loss, grad.astype(np.float64)


def host_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, int(os.environ.get("OMP_NUM_THREADS", n))))


def make_loss_oracle_pool(n_points, K):
    import multiprocessing as mp
    global _LOSS_IN
    sig = tuple(float(x) for x in np.asarray(synth.SIGMA_GRID, np.float32))
    _LOSS_IN = (synth.random_shading(n_points, K, seed=31), synth.random_materials(n_points, seed=32),
                synth.random_observations(n_points, seed=33), sig)
    w = host_workers()
    return mp.get_context("fork").Pool(w), w


def loss_oracle_leg(pool, workers, dev):
    """The numpy float64 loss+gradient oracle over the synthetic room-sized
    point set, single-process and on all host cores, and the accuracy of the
    GPU kernel and of the plain torch-autograd comparator (float32 and
    float64) against it on the same inputs."""
    from oracle import render as orr
    sh, mat, obs, sig = _LOSS_IN
    n = mat.shape[1]
    t0 = time.perf_counter()
    loss_o, grad_o, _ = orr.loss_and_grad(sh, mat, obs, sig)
    t_single = time.perf_counter() - t0
    edges = np.linspace(0, n, 4 * workers + 1).astype(np.int64)
    t0 = time.perf_counter()
    parts = pool.map(_loss_chunk, list(zip(edges[:-1], edges[1:])))
    t_all = time.perf_counter() - t0
    loss_p = math.fsum(p[0] for p in parts)
    grad_p = np.concatenate([p[1] for p in parts], axis=1)
    assert abs(loss_p - loss_o) <= 1e-12 * abs(loss_o) and np.array_equal(grad_p, grad_o)
    S, M, O = (torch.from_numpy(x).to(dev) for x in (sh, mat, obs))
    tau = 1e-6 * np.abs(grad_o).max(axis=1, keepdims=True)

    def err(loss, grad):
        g = grad.detach().double().cpu().numpy()
        return dict(loss_rel=abs(float(loss) - loss_o) / abs(loss_o),
                    grad_max_rel=float((np.abs(g - grad_o) / np.maximum(np.abs(grad_o), tau)).max()))

    buf, g_k, _ = fipt.fipt_render_loss(S, M, O, sig)
    acc = {"k_render_loss": err(buf[0].item(), g_k)}
    for dt, name in ((torch.float32, "torch_autograd_fp32"), (torch.float64, "torch_autograd_fp64")):
        l_t, g_t = torch_factored_loss(S, M, O, sig, dt)
        acc[name] = err(l_t.item(), g_t)
    for v in acc.values():
        v["meets_1e-4"] = v["grad_max_rel"] <= 1e-4 and v["loss_rel"] <= 1e-6
    del S, M, O
    return dict(points=n, single_process_s=t_single, all_cores_s=t_all, processes=workers,
                points_per_s_single=n / t_single, points_per_s_all_cores=n / t_all,
                accuracy_vs_oracle=acc,
                inputs="synthetic: shading U-shaped per level, materials uniform (roughness "
                       "touches every level), observations uniform; 1,843,200 points")


def torch_factored_loss(shading, material, observed, sigma, dtype):
    """The plain method: Eq. 5 with the lerp of Eq. 8 and the L2 loss of
    Eq. 2 as a torch expression in `dtype`, its gradient with respect to the
    material by autograd.  Same clamping as the kernel: t is clamped to
    [0, 1] (zero roughness gradient outside the level table)."""
    K = len(sigma)
    N = material.shape[1]
    g = torch.tensor(sigma, dtype=dtype, device=material.device)
    m = material.detach().to(dtype).requires_grad_(True)
    a, s, met = m[0:3], m[3], m[4]
    j = (torch.searchsorted(g, s.detach().contiguous(), right=True) - 1).clamp_(0, K - 2)
    t = ((s - g[j]) / (g[j + 1] - g[j])).clamp(0.0, 1.0)
    sh = shading.to(dtype)
    Ld = sh[0:3]
    L0s = sh[3:3 + 3 * K].view(K, 3, N)
    L1s = sh[3 + 3 * K:3 + 6 * K].view(K, 3, N)
    i0 = j.view(1, 1, N).expand(1, 3, N)
    L0 = (1.0 - t) * L0s.gather(0, i0)[0] + t * L0s.gather(0, i0 + 1)[0]
    L1 = (1.0 - t) * L1s.gather(0, i0)[0] + t * L1s.gather(0, i0 + 1)[0]
    kd = a * (1.0 - met)
    ks = 0.04 * (1.0 - met) + a * met
    Lr = kd * Ld + ks * L0 + L1
    loss = ((Lr - observed.to(dtype)) ** 2).sum()
    grad, = torch.autograd.grad(loss, m)
    return loss, grad


def run_comparator(shading, mat, obs, sigma, t_kernel_ms, reps=10):
    """The hand-written fused kernel against the plain torch-autograd
    expression of the same loss, on the same inputs and stream: forward +
    backward time, float32 and float64 (the kernel's own arithmetic)."""
    N = mat.shape[1]
    out = {"points": N, "k_render_loss_ms": t_kernel_ms,
           "k_render_loss_points_per_s": N / (t_kernel_ms * 1e-3)}
    for dt, name in ((torch.float32, "torch_autograd_fp32"), (torch.float64, "torch_autograd_fp64")):
        torch_factored_loss(shading, mat, obs, sigma, dt)
        torch.cuda.synchronize()
        tm = Timer()
        for _ in range(reps):
            tm.mark("a")
            torch_factored_loss(shading, mat, obs, sigma, dt)
            tm.mark("b")
        torch.cuda.synchronize()
        ms = float(np.mean(tm.spans("a", "b")))
        out[name] = {"ms": ms, "points_per_s": N / (ms * 1e-3), "kernel_speedup": ms / t_kernel_ms}
    out["note"] = ("accuracy of each against the float64 oracle on a room-sized synthetic set: "
                   "cpu_baseline.loss_grad.accuracy_vs_oracle")
    return out


def serving_setup(dev):
    """Eight resident rooms (18,860 ... 1,980,160 triangles) and their camera
    points."""
    rooms = synth.serving_rooms()
    scenes, pts = [], []
    for r in rooms:
        s = setup_room(r, dev)
        planes, tri = fipt.fipt_gen_points(s, r.cameras)
        scenes.append(s)
        pts.append((planes, tri))
    torch.cuda.synchronize()
    return rooms, scenes, pts


def trace_samples(trace):
    return sum(q["count"] * q["spp"] * (1 + len(synth.SIGMA_GRID)) for q in trace)


def serve_batched(scenes, pts, trace, log_every=20, tag="serving"):
    """Replay ``trace`` through the continuous-batching server; latency =
    completion - submission (at the request's arrival time)."""
    sig = synth.SIGMA_GRID
    srv = fipt.Server(device=0, pool_bytes=8 << 30, max_inflight=64, samples_per_launch=1 << 26)
    t0 = time.perf_counter()
    tickets = [None] * len(trace)

    def feeder():
        for i, q in enumerate(trace):
            d = t0 + q["arrival"] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            planes, tri = pts[q["room"]]
            tickets[i] = srv.submit(scenes[q["room"]], planes, tri, q["spp"], q["spp"], sig,
                                    q["seed"], offset=q["offset"], count=q["count"])

    th = threading.Thread(target=feeder)
    th.start()
    lat = []
    for i in range(len(trace)):
        while tickets[i] is None:
            time.sleep(1e-4)
        t = tickets[i]
        srv.wait(t)
        res = srv.result(t, copy=False)
        lat.append((res.t_done_us - res.t_submit_us) / 1e3)
        srv.release(t)
        if (i + 1) % log_every == 0:
            log(f"{tag}: {i + 1}/{len(trace)} requests done")
    th.join()
    makespan = time.perf_counter() - t0
    st = srv.stats()
    srv.destroy()
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                makespan_s=makespan, gsamples_per_s=trace_samples(trace) / makespan / 1e9,
                launches=int(st.launches), tiles=int(st.tiles))


def serve_single(scenes, pts, trace, log_every=20, tag="one-at-a-time"):
    """The same trace served one request at a time, FIFO, with fipt_bake."""
    sig = synth.SIGMA_GRID
    out = torch.empty((SHADING_PLANES, max(q["count"] for q in trace)), dtype=torch.float32,
                      device=pts[0][0].device)
    lat = []
    t0 = time.perf_counter()
    for i, q in enumerate(trace):
        d = t0 + q["arrival"] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        planes, tri = pts[q["room"]]
        o, c = q["offset"], q["count"]
        fipt.fipt_bake(scenes[q["room"]], planes[:, o:o + c].contiguous(), tri[o:o + c].contiguous(),
                       q["spp"], q["spp"], sig, q["seed"], out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - (t0 + q["arrival"])) * 1e3)
        if (i + 1) % log_every == 0:
            log(f"{tag}: {i + 1}/{len(trace)} requests done")
    makespan = time.perf_counter() - t0
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                makespan_s=makespan, gsamples_per_s=trace_samples(trace) / makespan / 1e9)


def run_serving(dev, n_requests, load, n_burst=100, log_every=50):
    """Serving below capacity: the capacity of the server is measured with
    ``n_burst`` requests arriving at once, then a Poisson trace of
    ``n_requests`` requests at ``load`` x that rate (rooms, point counts and
    sample counts as the serving workload draws them) is replayed through the
    server and, separately, one request at a time."""
    rooms, scenes, pts = serving_setup(dev)
    sizes = [p[0].shape[1] for p in pts]
    burst = synth.serving_trace(n_burst, 1e9, sizes, seed=1105)
    cap = serve_batched(scenes, pts, burst, log_every, "capacity")
    cap_rps = n_burst / cap["makespan_s"]
    rate = load * cap_rps
    log(f"serving capacity {cap_rps:.1f} requests/s; trace at {rate:.1f} requests/s")
    trace = synth.serving_trace(n_requests, rate, sizes, seed=1106)
    batched = serve_batched(scenes, pts, trace, log_every)
    single = serve_single(scenes, pts, trace, log_every)
    for s in scenes:
        s.destroy()
    p99 = batched["p99_ms"] / single["p99_ms"]
    return dict(requests=len(trace), load=load, rate_per_s=rate, rooms=[r.n_tris for r in rooms],
                capacity=dict(requests=n_burst, requests_per_s=cap_rps,
                              gsamples_per_s=cap["gsamples_per_s"]),
                lobe_samples=trace_samples(trace), batched=batched, one_at_a_time=single,
                p50_ratio_batched_to_single=batched["p50_ms"] / single["p50_ms"],
                p99_ratio_batched_to_single=p99,
                summary=("batched p99 more than 2 % below one-at-a-time" if p99 < 0.98 else
                         "batched p99 within 2 % of one-at-a-time (continuous batching lowers "
                         "the median, not the tail, at this load)" if p99 <= 1.02 else
                         "batched p99 ABOVE one-at-a-time"))


def serving_study(dev, n_trace, rate, n_sweep):
    """Capacity (all requests arriving at once), the Poisson trace at
    ``rate``, and a rate sweep at 0.5, 0.7 and 0.9 of capacity; each served
    batched and one at a time."""
    rooms, scenes, pts = serving_setup(dev)
    sizes = [p[0].shape[1] for p in pts]
    burst = synth.serving_trace(n_sweep, 1e9, sizes, seed=1105)
    cap = serve_batched(scenes, pts, burst, 50, "capacity")
    cap_rps = n_sweep / cap["makespan_s"]
    log(f"capacity: {cap_rps:.1f} requests/s, {cap['gsamples_per_s']:.2f} Gsamples/s")
    trace = synth.serving_trace(n_trace, rate, sizes)
    main_b = serve_batched(scenes, pts, trace, 100, f"rate {rate:g}")
    main_s = serve_single(scenes, pts, trace, 100, f"rate {rate:g} one-at-a-time")
    sweep = []
    for f in (0.5, 0.7, 0.9):
        r = f * cap_rps
        tr = synth.serving_trace(n_sweep, r, sizes, seed=1106)
        b = serve_batched(scenes, pts, tr, 100, f"{f:g} x capacity")
        s1 = serve_single(scenes, pts, tr, 100, f"{f:g} x capacity one-at-a-time")
        sweep.append(dict(load=f, rate_per_s=r, requests=n_sweep, lobe_samples=trace_samples(tr),
                          batched=b, one_at_a_time=s1))
    for s in scenes:
        s.destroy()
    return dict(rooms=[r.n_tris for r in rooms],
                capacity=dict(requests=n_sweep, requests_per_s=cap_rps, **cap),
                trace=dict(requests=n_trace, rate_per_s=rate, lobe_samples=trace_samples(trace),
                           batched=main_b, one_at_a_time=main_s),
                sweep=sweep)


def bake_roofline(trav, t_bake_ms, traffic):
    """Roofline of one bake launch: algorithmic flops (counted from the
    instrumented twin of the kernel) over the launch time, against the
    published FP32 vector peak; the issue-rate view and the traversal bytes
    as secondary figures."""
    tf = trav["flops"] / (t_bake_ms * 1e-3) / 1e12
    tops = trav["ops"] / (t_bake_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / PEAK_FP32_TFLOPS, "traffic": traffic, "kernel": "k_bake",
            "flops_per_launch": trav["flops"],
            "flops_counted": "20 per ray-box test (80 per 4-wide node visited, 60 per chain "
                             "level: the three siblings of the point's chain child), 30 per "
                             "ray-triangle test, 100 per lobe sample",
            "issue_rate": {"achieved_tops": tops, "peak_tops": PEAK_VALU_TOPS,
                           "frac": tops / PEAK_VALU_TOPS, "ops_per_launch": trav["ops"],
                           "note": "VALU operations counted per instruction against one "
                                   "operation per lane per cycle (no packed FP32)"},
            "effective_traversal_gbs": trav["bytes"] / (t_bake_ms * 1e-3) / 1e9,
            "traversal_bytes_per_launch": trav["bytes"],
            "traversal_note": "bytes the node, triangle and radiance loads request, mostly "
                              "served from L1/L2/MALL: not an HBM roofline"}


def hbm_bandwidth(dev, n=1 << 28, reps=5):
    """Achievable HBM bandwidth from the library's streaming kernel
    (fipt_hbm_stream) on 1 GiB float arrays: copy (8 bytes per element) and
    triad (12 bytes per element), best of the two; torch's copy_ beside it."""
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.ones(n, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    res = {}
    for kind, name, per in ((0, "copy", 8), (1, "triad", 12)):
        fipt.fipt_hbm_stream(kind, a, c, b, 0.5)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fipt.fipt_hbm_stream(kind, a, c, b, 0.5)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"{name}_ms"] = ms
        res[f"{name}_gbs"] = per * n / (ms * 1e-3) / 1e9
    del a, b, c
    res["torch_copy_gbs"], _ = copy_bandwidth(dev, n, reps)
    res["bytes"] = {"copy": 8 * n, "triad": 12 * n}
    res["achievable_gbs"] = max(res["copy_gbs"], res["triad_gbs"])
    return res


def copy_bandwidth(dev, n=1 << 28, reps=5):
    """A 1 GiB float32 device-to-device copy by torch (copy_)."""
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return 8 * n / (ms * 1e-3) / 1e9, ms


def loss_timing(shading, mat, obs, sigma, reps=10, flush=None, alpha=None, lambda_d=0.0,
                tonemap=0):
    """Mean fused render + loss + gradient time (ms) over ``reps`` launches;
    with ``flush`` (a >= 512 MB tensor) the caches are refilled by reading it
    before each launch (reads, so no dirty lines are left to write back), and
    the kernel's inputs come from HBM.  With ``alpha`` the emission-masked
    loss with the diffuse prior is timed (material and mask gradients)."""
    n = shading.shape[1]
    grad = torch.empty((5, n), dtype=torch.float32, device=shading.device)
    buf = torch.empty((fipt.LOSS_SLOTS,), dtype=torch.float64, device=shading.device)
    galpha = torch.empty((n,), dtype=torch.float32, device=shading.device)

    def launch():
        if alpha is None:
            fipt.fipt_render_loss(shading, mat, obs, sigma, tonemap, loss_buf=buf, grad=grad)
        else:
            fipt.fipt_render_loss_masked(shading, mat, obs, sigma, alpha, lambda_d, tonemap,
                                         loss_buf=buf, grad=grad, grad_alpha=galpha)

    launch()
    # a ~2 ms spin first, so the host has queued the launches before the GPU
    # reaches them and the events time the kernels, not the Python calls
    torch.cuda._sleep(5_000_000)
    tm = Timer()
    for _ in range(reps):
        if flush is not None:
            flush.sum()
        tm.mark("a")
        launch()
        tm.mark("b")
    torch.cuda.synchronize()
    return float(np.mean(tm.spans("a", "b")))


def run_voxel(scene, sc, planes, tri, obs, out, reps=3):
    """The radiance cache as Sec. 4.2 builds it, on the room: the
    observations pooled onto a 256^3 voxel grid over the room's box, then
    bakes whose radiance query reads the voxel of each hit (plus the
    triangles' emission).  The scene's own cache is restored afterwards."""
    R = VOXEL_RES
    N = planes.shape[1]
    S = sc.spp * (1 + len(sc.sigma))
    bmin, bmax = sc.bmin.tolist(), sc.bmax.tolist()
    t0 = time.perf_counter()
    plan = fipt.VoxelPlan(planes[0:3].cpu().numpy(), R, bmin, bmax)
    plan_s = time.perf_counter() - t0
    cache = plan.pool(obs)
    torch.cuda.synchronize()
    torch.cuda._sleep(5_000_000)
    tm = Timer()
    for _ in range(reps):
        tm.mark("a")
        plan.pool(obs, out=cache)
        tm.mark("b")
    torch.cuda.synchronize()
    t_pool = float(np.mean(tm.spans("a", "b")))
    occupied = int((cache.abs().sum(0) > 0).sum().item())
    em = torch.from_numpy(sc.emission).to(obs.device)
    scene.set_voxel_radiance(cache, R, bmin, bmax, em)
    fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=out)
    torch.cuda.synchronize()
    tb = Timer()
    for _ in range(reps):
        tb.mark("a")
        fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=out)
        tb.mark("b")
    torch.cuda.synchronize()
    t_bake = float(np.mean(tb.spans("a", "b")))
    kind = fipt.CACHE_VERTEX if sc.cache_kind == "vertex" else fipt.CACHE_TRIANGLE
    scene.set_radiance(torch.from_numpy(sc.cache).to(obs.device), kind, em)
    torch.cuda.synchronize()
    pool_bytes = 16 * (R ** 3 + N)
    del plan, cache
    return {"res": R, "kernel": "k_bake<false, true, true>",
            "traffic": measured_traffic().get("k_bake_voxel"), "plan_build_s": plan_s, "pool_ms": t_pool, "pool_bytes": pool_bytes,
            "pool_gbs": pool_bytes / (t_pool * 1e-3) / 1e9, "occupied_voxels": occupied,
            "bake_ms": t_bake, "gsamples_per_s": N * S / (t_bake * 1e-3) / 1e9,
            "note": "pool bytes: start index and output per voxel (4 + 12 B), order index and "
                    "observation per pixel (4 + 12 B)"}


def run_refine(scene, sc, planes, tri, grid, out, t_bake_ms, reps=3):
    """The stage-3 refinement (Eq. 10 / 11) of the room's shadings under the
    current material (the differentiation workload's 128^3 grid): paths
    grown through glossy hits (roughness <= 0.6) to an emitter or a rough
    hit, at most eight vertices, emitter sampling with MIS at glossy
    vertices; same points and lobe samples as the bake."""
    N = planes.shape[1]
    S = sc.spp * (1 + len(sc.sigma))
    bmin, bmax = sc.bmin.tolist(), sc.bmax.tolist()

    def once():
        fipt.fipt_refine(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, grid, bmin, bmax,
                         out=out)

    once()
    torch.cuda.synchronize()
    tm = Timer()
    for _ in range(reps):
        tm.mark("a")
        once()
        tm.mark("b")
    torch.cuda.synchronize()
    ms = float(np.mean(tm.spans("a", "b")))
    glossy = float((grid[3] <= 0.6).float().mean().item())
    return {"points": N, "lobe_samples_per_point": S, "max_vertices": 8, "sigma_diffuse": 0.6,
            "ms": ms, "gsamples_per_s": N * S / (ms * 1e-3) / 1e9, "bake_ms": t_bake_ms,
            "cost_vs_bake": ms / t_bake_ms, "kernel": "k_refine",
            "material": "differentiation workload's 128^3 grid (roughness U[0.02, 1] per node; "
                        f"{glossy:.0%} of nodes glossy)"}


def run_hashgrid(sc, planes, shading, obs, reps=5):
    """The paper's material network (Eq. 14) on the room's points: a training
    step (the forward pass keeping the encoding, the factored loss with its
    material gradient, the backward pass into table and weight gradients
    reading the kept encoding), and the plain forward pass alone."""
    N = planes.shape[1]
    dev = planes.device
    bmin, bmax = sc.bmin.tolist(), sc.bmax.tolist()
    params = torch.from_numpy(synth.hashgrid_params()).to(dev)
    pos = planes[0:3].contiguous()
    mat = torch.empty((5, N), dtype=torch.float32, device=dev)
    gmat = torch.empty((5, N), dtype=torch.float32, device=dev)
    gpar = torch.zeros_like(params)
    ws = torch.empty((int(fipt.lib().fipt_hashgrid_workspace_floats(N)),), dtype=torch.float32,
                     device=dev)
    buf = torch.empty((fipt.LOSS_SLOTS,), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = fipt.HashGridPlan(pos, bmin, bmax)   # once per point set
    t_plan = time.perf_counter() - t0

    def once(tm=None):
        if tm:
            tm.mark("a")
        fipt.fipt_hashgrid_forward_save(params, plan, ws, out=mat)
        if tm:
            tm.mark("b")
        fipt.fipt_render_loss(shading, mat, obs, sc.sigma, loss_buf=buf, grad=gmat)
        if tm:
            tm.mark("c")
        gpar.zero_()
        if tm:
            tm.mark("d")
        fipt.fipt_hashgrid_backward(plan, params, gmat, grad_params=gpar, workspace=ws, saved=True)
        if tm:
            tm.mark("e")

    once()
    torch.cuda.synchronize()
    first = gpar.clone()
    torch.cuda._sleep(5_000_000)
    tm = Timer()
    for _ in range(reps):
        once(tm)
    torch.cuda.synchronize()
    repeatable = bool(torch.equal(first, gpar))
    # the plain forward pass (inference: nothing kept)
    tf = Timer()
    torch.cuda._sleep(5_000_000)
    for _ in range(reps):
        tf.mark("a")
        fipt.fipt_hashgrid_forward(params, pos, bmin, bmax, out=mat)
        tf.mark("b")
    torch.cuda.synchronize()
    t_fwd_plain = float(np.mean(tf.spans("a", "b")))
    del plan
    t_fwd = float(np.mean(tm.spans("a", "b")))
    t_loss = float(np.mean(tm.spans("b", "c")))
    t_zero = float(np.mean(tm.spans("c", "d")))
    t_bwd = float(np.mean(tm.spans("d", "e")))
    # vertex reads the forward pass needs: a vertex with zero trilinear weight
    # is not read (from level 20 on a single-precision position sits on a
    # vertex); counted from the same single-precision cell arithmetic
    lo = torch.tensor(bmin, dtype=torch.float32, device=dev)[:, None]
    inv = 1.0 / (torch.tensor(bmax, dtype=torch.float32, device=dev)[:, None] - lo)
    p = torch.clamp((pos - lo) * inv, 0.0, 1.0)
    reads = torch.zeros(N, dtype=torch.float64, device=dev)
    for lv in range(32):
        nl = float(16 * 2 ** lv)
        u = p * nl
        f = u - torch.minimum(torch.floor(u), torch.full_like(u, nl - 1.0))
        reads += torch.prod(1.0 + (f != 0).to(torch.float64), dim=0)
    reads_pp = float(reads.mean().item())
    bytes_pp = 8.0 * reads_pp + 32.0
    # the backward call's algorithmic bytes per point: the per-point kernel
    # (the kept encoding and the output gradient in, 261 activations and
    # layer gradients and 64 feature gradients out), the table gather (an
    # 8-byte entry and an 8-byte feature gradient per nonzero (point, corner),
    # as many as the forward's vertex reads), the weight-gradient products
    # (the 325 workspace floats read once); the tables' read-modify-write of
    # touched slots is not counted
    bwd_pp = 4.0 * 64 + 20.0 + 4.0 * (261 + 64) + 16.0 * reads_pp + 4.0 * 325
    bwd_note = ("4 B x 64 encoding + 20 B in, 4 B x (261 + 64) out (per-point kernel); 16 B x vertex "
                "reads (table gather); 4 B x 325 (weight-gradient products); table read-modify-write "
                "not counted")
    del p, u, f, reads
    fwd_gbs = bytes_pp * N / (t_fwd_plain * 1e-3) / 1e9
    return {"points": N, "params": int(params.numel()), "forward_ms": t_fwd_plain,
            "step": "fipt_hashgrid_forward_save (the encoding kept, 256 B per point more written) + "
                    "loss + fipt_hashgrid_backward_saved",
            "forward_save_ms": t_fwd,
            "traffic_forward_save": measured_traffic().get("k_hg_forward_save"),
            "loss_ms": t_loss, "zero_grad_ms": t_zero, "backward_ms": t_bwd,
            "backward_bitwise_repeatable": repeatable, "table_gradient": "gather over a per-level "
            "slot-sorted (point, corner) list (no atomics)", "plan_build_s": t_plan,
            "step_points_per_s": N / ((t_fwd + t_loss + t_zero + t_bwd) * 1e-3),
            "forward_vertex_reads_per_point": reads_pp,
            "forward_bytes_per_point": bytes_pp,
            "forward_gbs": fwd_gbs,
            "forward_flops_per_point": HG_FWD_FLOPS_PER_POINT,
            "forward_tflops": HG_FWD_FLOPS_PER_POINT * N / (t_fwd_plain * 1e-3) / 1e12,
            "traffic_forward": measured_traffic().get("k_hg_forward"),
            "kernel": "k_hg_forward",
            "roofline_forward": {"bound": "hbm", "achieved": fwd_gbs,
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": fwd_gbs / PEAK_HBM_GBS,
                                 "traffic": measured_traffic().get("k_hg_forward"),
                                 "kernel": "k_hg_forward"},
            "backward_bytes_per_point": bwd_pp,
            "backward_bytes_note": bwd_note,
            "roofline_backward": {"bound": "hbm", "achieved": bwd_pp * N / (t_bwd * 1e-3) / 1e9,
                                  "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": bwd_pp * N / (t_bwd * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                  "traffic": measured_traffic().get("k_hg_backward"),
                                  "kernel": "k_hg_backward + k_hg_table_grad + k_hg_wgrad + k_hg_wreduce"}}


def run_large(dev, rebakes, copy_gbs):
    """The emitter loop on the ~2M-triangle room: ``rebakes`` iterations,
    each re-estimating the per-triangle emission of that iteration's emitter
    triangles as the median of their pixels' observations (Eq. 13 with
    f = 0), uploading it and baking 1,000,000 points x 256 spp x 7 lobes;
    then the fused loss + gradient on the last bake's shadings."""
    t0 = time.perf_counter()
    sc = synth.large_room()
    scene = setup_room(sc, dev)
    planes, tri = fipt.fipt_gen_points(scene, sc.cameras)
    N = planes.shape[1]
    K = len(sc.sigma)
    S = sc.spp * (1 + K)
    tri_host = tri.cpu().numpy()
    sched = [torch.from_numpy(f.astype(np.uint8)).to(dev) for f in synth.emitter_schedule(sc.emission, rebakes)]
    obs_em = torch.from_numpy(synth.emitter_observations(sc.emission, tri_host)).to(dev)
    eplan = fipt.EmissionPlan(tri_host, sc.n_tris)
    le = torch.empty((3, sc.n_tris), dtype=torch.float32, device=dev)
    eplan.median(obs_em, sched[0], out=le)                                           # warm-up
    out = torch.empty((3 + 6 * K, N), dtype=torch.float32, device=dev)
    fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=out)   # warm-up
    torch.cuda.synchronize()
    log(f"large room setup {time.perf_counter() - t0:.1f} s: {sc.n_tris} triangles, {N} points")
    tm = Timer()
    t1 = time.perf_counter()
    for i, flags in enumerate(sched):
        tm.mark("a")
        eplan.median(obs_em, flags, out=le)
        tm.mark("b")
        scene.set_emission(le)
        tm.mark("c")
        fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=out)
        tm.mark("d")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    log(f"large room: {rebakes} re-bakes in {wall:.2f} s")
    t_bake = float(np.mean(tm.spans("c", "d")))
    t_median = float(np.mean(tm.spans("a", "b")))
    t_emis = float(np.mean(tm.spans("b", "c")))
    n_emitters = int(sched[-1].sum())
    del eplan
    trav = traversal_bytes(scene, planes, tri, sc, out)
    # material gathered from a 128^3 grid over the room (as in the
    # differentiation workload), observations synthetic
    grid = torch.from_numpy(synth.material_grid(128, seed=1007)).to(dev)
    mat = fipt.fipt_grid_gather(grid, sc.bmin.tolist(), sc.bmax.tolist(), planes[0:3].contiguous())
    obs = torch.from_numpy(synth.random_observations(N)).to(dev)
    flush = torch.ones((1 << 27,), dtype=torch.float32, device=dev)      # 512 MB
    t_warm = loss_timing(out, mat, obs, sc.sigma)
    t_cold = loss_timing(out, mat, obs, sc.sigma, flush=flush)
    # the fused step (material fetch, render, loss, adjoint) on the same
    # shadings put into the grid plan's order
    plan = fipt.GridPlan(planes[0:3].cpu().numpy(), 128, sc.bmin.tolist(), sc.bmax.tolist())
    out_q, obs_q = plan.permute(out), plan.permute(obs)
    gg = torch.empty_like(grid)
    lb = torch.empty((fipt.LOSS_SLOTS,), dtype=torch.float64, device=dev)
    fused = {}
    plan.render_loss(grid, out_q, obs_q, sc.sigma, loss_buf=lb, grad_grid=gg)
    for name, fl in (("warm", None), ("cold", flush)):
        ts = []
        torch.cuda._sleep(5_000_000)     # the host queues the launches ahead of the GPU
        for _ in range(10):
            if fl is not None:
                fl.sum()                                  # evicts L2 and the MALL
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record()
            plan.render_loss(grid, out_q, obs_q, sc.sigma, loss_buf=lb, grad_grid=gg)
            s1.record()
            ts.append((s0, s1))
        torch.cuda.synchronize()
        fused[name] = float(np.median([a.elapsed_time(b) for a, b in ts]))
    fused_bytes = N * FUSED_LOSS_BYTES_PER_POINT + 2 * 5 * 128 ** 3 * 4
    del flush, plan, out_q, obs_q
    scene.destroy()
    gbs = lambda ms: N * LOSS_BYTES_PER_POINT / (ms * 1e-3) / 1e9
    eff = trav["bytes"] / (t_bake * 1e-3) / 1e9
    roof = bake_roofline(trav, t_bake, None)
    return {
        "workload": f"large room: {sc.n_tris:,} triangles, {len(sc.cameras)} cameras x 250x250 = "
                    f"{N:,} points, {sc.spp} spp per lobe, {K} roughness levels, {rebakes} re-bakes, "
                    "each after re-estimating the emitters' per-triangle emission as the median of "
                    "their pixels' observations",
        "rebakes": rebakes,
        "ms_per_rebake": wall * 1e3 / rebakes,
        "bake_ms": t_bake,
        "emission_median_ms": t_median,
        "emitter_triangles": n_emitters,
        "set_emission_ms": t_emis,
        "gsamples_per_s": N * S / (t_bake * 1e-3) / 1e9,
        "rays_per_s": trav["rays"] / (t_bake * 1e-3),
        "traversal": trav,
        "roofline": roof,
        "roofline_loss": {"bound": "hbm", "achieved": gbs(t_warm), "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": gbs(t_warm) / PEAK_HBM_GBS, "traffic": None,
                          "bytes_per_point": LOSS_BYTES_PER_POINT, "kernel": "k_render_loss",
                          "cold": {"achieved": gbs(t_cold), "frac": gbs(t_cold) / PEAK_HBM_GBS}},
        "loss_grad": {"points": N, "warm_ms": t_warm, "cold_ms": t_cold,
                      "warm_gbs": gbs(t_warm), "cold_gbs": gbs(t_cold),
                      "warm_frac_of_achievable_hbm": gbs(t_warm) / copy_gbs,
                      "cold_frac_of_achievable_hbm": gbs(t_cold) / copy_gbs,
                      "bytes_per_point": LOSS_BYTES_PER_POINT,
                      "material": "gathered from a 128^3 grid (spatially coherent roughness)"},
        "fused_loss_grad": {"kernels": "fipt_grid_render_loss (material fetch + render + loss + "
                                       "grid adjoint, points in the plan's order)",
                            "warm_ms": fused["warm"], "cold_ms": fused["cold"],
                            "points_per_s": N / (fused["warm"] * 1e-3),
                            "roofline": {"bound": "hbm",
                                         "achieved": fused_bytes / (fused["warm"] * 1e-3) / 1e9,
                                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                         "frac": fused_bytes / (fused["warm"] * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                         "bytes_per_launch": fused_bytes, "traffic": None}},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--cpu-large-budget-s", type=float, default=12.0,
                    help="oracle budget on the 2M-triangle room (0 skips it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=300)
    ap.add_argument("--serving-load", type=float, default=0.9,
                    help="offered load of the serving trace as a fraction of measured capacity")
    ap.add_argument("--serving-rate", type=float, default=200.0,
                    help="arrival rate of the --serving-study trace")
    ap.add_argument("--no-counters", action="store_true")
    ap.add_argument("--serving-study", action="store_true",
                    help="only run the serving study (capacity, the --serving-trace-requests "
                         "trace at --serving-rate, a load sweep) and print its JSON")
    ap.add_argument("--serving-trace-requests", type=int, default=2000)
    ap.add_argument("--serving-sweep-requests", type=int, default=300)
    ap.add_argument("--large-rebakes", type=int, default=10,
                    help="re-bakes of the ~2M-triangle emitter loop (0 skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 1 GiB device-to-device copies (counter scaling and "
                         "achievable HBM bandwidth) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the hot path has no multi-GPU leg); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    room_points = 24 * 320 * 240
    pool = workers = None
    if not args.no_cpu and not (args.copy_calibration or args.serving_study):
        # forked before anything touches the GPU
        pool, workers = make_loss_oracle_pool(room_points, len(synth.SIGMA_GRID))
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = 1 << 28                                      # 1 GiB of float32
        gbs, ms = copy_bandwidth(dev, n)
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                          "copy_ms": ms, "copy_gbs": gbs}), flush=True)
        return
    if args.serving_study:
        print(json.dumps(serving_study(dev, args.serving_trace_requests, args.serving_rate,
                                       args.serving_sweep_requests)), flush=True)
        return
    hbm = hbm_bandwidth(dev)
    copy_gbs = hbm["achievable_gbs"]
    log(f"achievable HBM bandwidth (1 GiB streaming kernel): copy {hbm['copy_gbs']:.0f} GB/s, "
        f"triad {hbm['triad_gbs']:.0f} GB/s; torch copy_ {hbm['torch_copy_gbs']:.0f} GB/s")

    t_setup = time.perf_counter()
    sc = synth.room()
    scene = setup_room(sc, dev)
    N = sc.n_points
    assert N == room_points
    K = len(sc.sigma)
    P = 3 + 6 * K
    S = sc.spp * (1 + K)
    planes, tri = fipt.fipt_gen_points(scene, sc.cameras)
    shading = torch.empty((P, N), dtype=torch.float32, device=dev)
    R = 128
    bmin, bmax = sc.bmin.tolist(), sc.bmax.tolist()
    grid_gt = torch.from_numpy(synth.material_grid(R, seed=1003)).to(dev)
    grid = torch.from_numpy(synth.material_grid(R, seed=1006)).to(dev)
    plan = fipt.GridPlan(planes[0:3].cpu().numpy(), R, bmin, bmax)
    # observations: factored render of the hidden material x (1 + 1% noise)
    fipt.fipt_bake(scene, planes, tri, sc.spp, sc.spp, sc.sigma, sc.seed, out=shading)
    mat_gt = fipt.fipt_grid_gather(grid_gt, bmin, bmax, planes[0:3].contiguous())
    zeros = torch.zeros((3, N), dtype=torch.float32, device=dev)
    _, _, lr_gt = fipt.fipt_render_loss(shading, mat_gt, zeros, sc.sigma, want_grad=False,
                                        want_lr=True)
    noise = torch.from_numpy(synth.observation_noise(N)).to(dev)
    obs = (lr_gt * (1.0 + 0.01 * noise)).contiguous()
    pos = planes[0:3].contiguous()
    mat = torch.empty((5, N), dtype=torch.float32, device=dev)
    grad_pts = torch.empty((5, N), dtype=torch.float32, device=dev)
    grad_grid = torch.empty_like(grid)
    loss_buf = torch.empty((fipt.LOSS_SLOTS,), dtype=torch.float64, device=dev)
    # the step works on the points in the grid plan's order (by node brick,
    # cell, index): the generated points are put into that order before the
    # bake, the observations once here, so the fused loss reads every
    # per-point plane contiguously and each workgroup's corners are local
    obs_q = plan.permute(obs)
    planes_q = torch.empty_like(planes)
    tri_q = torch.empty_like(tri)
    shading_q = torch.empty_like(shading)
    grad_grid_q = torch.empty_like(grid)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t_setup:.1f} s: {sc.n_tris} triangles, {N} points")

    tm = Timer()

    def step(timed):
        if timed:
            tm.mark("a")
        fipt.fipt_gen_points(scene, sc.cameras, planes=planes, tri=tri)
        plan.permute(planes, out=planes_q)
        plan.permute(tri.view(1, N), out=tri_q.view(1, N))
        if timed:
            tm.mark("b")
        fipt.fipt_bake(scene, planes_q, tri_q, sc.spp, sc.spp, sc.sigma, sc.seed, out=shading_q)
        if timed:
            tm.mark("c")
        plan.render_loss(grid, shading_q, obs_q, sc.sigma, loss_buf=loss_buf, grad_grid=grad_grid_q)
        if timed:
            tm.mark("d")

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_pts = float(np.mean(tm.spans("a", "b")))
    t_bake = float(np.mean(tm.spans("b", "c")))
    t_fused = float(np.mean(tm.spans("c", "d")))
    loss_value = float(loss_buf[0].item())
    # the same loss and gradient as three separate calls (gather, render-loss,
    # adjoint) on the points in camera order, timed alone
    sep = Timer()
    for i in range(args.steps + 1):
        sep.mark("c")
        fipt.fipt_grid_gather(grid, bmin, bmax, pos, out=mat)
        sep.mark("d")
        fipt.fipt_render_loss(shading, mat, obs, sc.sigma, loss_buf=loss_buf, grad=grad_pts)
        sep.mark("e")
        plan.scatter(grad_pts, out=grad_grid)
        sep.mark("f")
    torch.cuda.synchronize()
    t_gather = float(np.mean(sep.spans("c", "d")[1:]))
    t_loss = float(np.mean(sep.spans("d", "e")[1:]))
    t_scatter = float(np.mean(sep.spans("e", "f")[1:]))

    trav = None
    if not args.no_counters:
        # the timed bake's points: in the grid plan's order
        trav = traversal_bytes(scene, planes_q, tri_q, sc, torch.empty_like(shading))
        log(f"traversal: {trav}")
    loss_gbs = N * LOSS_BYTES_PER_POINT / (t_loss * 1e-3) / 1e9
    traffic = measured_traffic()
    # the material grid's gather and adjoint: each point reads its position
    # (12 B) and writes (gather) or reads (adjoint) five values (20 B); the
    # 5 x 128^3 grid is read once (gather) or written once (adjoint)
    grid_bytes = N * 32 + 5 * R ** 3 * 4
    fused_bytes = N * FUSED_LOSS_BYTES_PER_POINT + 2 * 5 * R ** 3 * 4
    roof_grid = {
        kname: {"bound": "hbm", "achieved": grid_bytes / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": grid_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "ms": ms, "bytes_per_launch": grid_bytes, "kernel": kn, "traffic": traffic.get(tk)}
        for kname, ms, kn, tk in (("gather", t_gather, "k_grid_gather", "k_grid_gather"),
                                  ("adjoint", t_scatter, "k_grid_adjoint + k_grid_adjoint_combine",
                                   "k_grid_adjoint"))}

    flush = torch.ones((1 << 27,), dtype=torch.float32, device=dev)      # 512 MB
    t_loss_cold = loss_timing(shading, mat, obs, sc.sigma, flush=flush)
    # the emission-masked loss with the diffuse prior (Eq. 15 + Eq. 17), with
    # and without the tone map, on a mask shaped by the room's emitters
    alpha = torch.from_numpy(synth.emission_mask(sc.emission, tri.cpu().numpy())).to(dev)
    masked = {"bytes_per_point": MASKED_LOSS_BYTES_PER_POINT, "lambda_d": LAMBDA_D,
              "traffic_log_srgb": traffic.get("k_render_loss_masked"),
              "mask": "0.5-1 on pixels of emissive triangles, below 0.02 elsewhere"}
    for tone, name in ((0, "identity"), (1, "log_srgb")):
        warm = loss_timing(shading, mat, obs, sc.sigma, alpha=alpha, lambda_d=LAMBDA_D,
                           tonemap=tone)
        cold = loss_timing(shading, mat, obs, sc.sigma, flush=flush, alpha=alpha,
                           lambda_d=LAMBDA_D, tonemap=tone)
        masked[name] = {"warm_ms": warm, "cold_ms": cold,
                        "warm_gbs": N * MASKED_LOSS_BYTES_PER_POINT / (warm * 1e-3) / 1e9,
                        "cold_gbs": N * MASKED_LOSS_BYTES_PER_POINT / (cold * 1e-3) / 1e9,
                        "points_per_s": N / (warm * 1e-3)}
    log(f"masked loss: {masked}")
    del flush, alpha
    comparator = run_comparator(shading, mat, obs, sc.sigma, t_loss)
    log(f"torch-autograd comparator: {comparator}")
    refine = run_refine(scene, sc, planes_q, tri_q, grid, torch.empty_like(shading), t_bake)
    log(f"stage-3 refinement: {refine}")
    voxel = run_voxel(scene, sc, planes, tri, obs, shading)
    log(f"voxel cache: {voxel}")
    # on the points in the grid plan's order, as the step keeps them (neighbouring
    # points share table lines: 7 % faster forward than in camera order)
    hashgrid = run_hashgrid(sc, planes_q, shading_q, obs_q)
    log(f"hash-grid network: {hashgrid}")

    large = None
    if args.large_rebakes > 0:
        large = run_large(dev, args.large_rebakes, copy_gbs)
        log(f"large room: {large['gsamples_per_s']:.2f} Gsamples/s, roofline "
            f"{large['roofline']['frac']:.3f} of the FP32 peak")

    cpu = None
    if pool is not None:
        log("cpu baseline: timing the oracle on bounded samples ...")
        loss_leg = loss_oracle_leg(pool, workers, dev)
        pool.close()
        pool.join()
        cpu = cpu_baseline(sc, args.cpu_budget_s,
                           synth.large_room() if args.cpu_large_budget_s > 0 else None,
                           args.cpu_large_budget_s, loss_leg)
        log(f"cpu baseline: {cpu}")

    serving = None
    if args.serving_requests > 0:
        serving = run_serving(dev, args.serving_requests, args.serving_load)

    out = {
        "metric": "Gsamples/s shading bake; factored loss+grad points/s; p50/p99 bake latency",
        "value": N * S / (ms_step * 1e-3) / 1e9,
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "room: 189,440 triangles, 24 cameras x 320x240 = 1,843,200 points, "
                               "128 spp per lobe, 6 roughness levels; 128^3 material grid",
                   "points": N, "lobe_samples_per_point": S, "triangles": sc.n_tris,
                   "parallelism": "single GPU"},
        "breakdown_ms": {"points_and_plan_order": t_pts, "bake": t_bake,
                         "fused_grid_loss_fwd_bwd": t_fused},
        "bake_gsamples_per_s": N * S / (t_bake * 1e-3) / 1e9,
        "loss_grad_points_per_s": N / (t_fused * 1e-3),
        "loss_grad": {"kernels": "k_grid_render_loss + k_grid_adjoint_sums (its last workgroup sums "
                                 "the loss) + k_grid_adjoint_combine (one call, points in the grid "
                                 "plan's order)",
                      "ms": t_fused, "points_per_s": N / (t_fused * 1e-3),
                      "roofline": {"bound": "hbm", "achieved": fused_bytes / (t_fused * 1e-3) / 1e9,
                                   "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": fused_bytes / (t_fused * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                   "bytes_per_launch": fused_bytes,
                                   "bytes_counted": "per point: position 12 B, Ld 12 B, the two "
                                                    "bracketing levels of Ls0 and Ls1 48 B, Lgt 12 B; "
                                                    "the 5 x 128^3 grid read once and its gradient "
                                                    "written once",
                                   "traffic": traffic.get("k_grid_render_loss")},
                      "separate_calls": {"grid_gather_ms": t_gather, "render_loss_ms": t_loss,
                                         "grid_scatter_ms": t_scatter,
                                         "points_per_s": N / ((t_loss + t_gather + t_scatter) * 1e-3),
                                         "note": "the same computation as three calls on the points "
                                                 "in camera order"}},
        "render_loss_points_per_s": N / (t_loss * 1e-3),
        "render_loss_gbs": loss_gbs,
        "render_loss_cold_ms": t_loss_cold,
        "render_loss_cold_gbs": N * LOSS_BYTES_PER_POINT / (t_loss_cold * 1e-3) / 1e9,
        "achievable_hbm_gbs": copy_gbs,
        "hbm_probe": hbm,
        "loss": loss_value,
        "traversal": trav,
        "roofline": bake_roofline(trav, t_bake, traffic.get("k_bake")) if trav else None,
        "roofline_render_loss": {"bound": "hbm", "achieved": loss_gbs, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": loss_gbs / PEAK_HBM_GBS,
                                 "traffic": traffic.get("k_render_loss"),
                                 "bytes_per_point": LOSS_BYTES_PER_POINT, "kernel": "k_render_loss",
                                 "frac_of_achievable": loss_gbs / copy_gbs,
                                 "cold": {"achieved": N * LOSS_BYTES_PER_POINT / (t_loss_cold * 1e-3) / 1e9,
                                          "frac": N * LOSS_BYTES_PER_POINT / (t_loss_cold * 1e-3) / 1e9 / PEAK_HBM_GBS}},
        "roofline_grid": roof_grid,
        "torch_autograd_comparator": comparator,
        "masked_loss": masked,
        "refinement": refine,
        "voxel_cache": voxel,
        "hashgrid_network": hashgrid,
        "cpu_baseline": cpu,
        "serving": serving,
        "large_room": large,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
