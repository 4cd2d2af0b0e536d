"""Parity criteria shared by the GPU tests.

Bake (float32 kernel vs float64 oracle):
  per value   rel = |gpu - oracle| / max(|oracle|, tau), tau = 1e-6 x the
              largest |oracle| of that output plane over the compared points;
  per point   the largest rel over its 3 + 6K values;
  pass        >= 99.9 % of points within 1e-4, and every other point either
              within 1e-2 or with all its values inside the oracle's
              envelope of single-precision-ambiguous ray outcomes widened
              by 1e-4 relative.
"""
import numpy as np


def plane_tau(oracle: np.ndarray, floor: float = 1e-6) -> np.ndarray:
    return floor * np.maximum(np.abs(oracle).max(axis=1, keepdims=True), 1e-30)


def bake_report(gpu: np.ndarray, res: dict) -> dict:
    o = res["mean"]
    g = gpu.astype(np.float64)
    tau = plane_tau(o)
    rel = np.abs(g - o) / np.maximum(np.abs(o), tau)
    per_point = rel.max(axis=0)
    lo, hi = res["lo"], res["hi"]
    slack = 1e-4 * np.maximum(np.abs(lo), np.abs(hi)) + tau
    inside = np.all((g >= lo - slack) & (g <= hi + slack), axis=0)
    n = per_point.size
    within = per_point <= 1e-4
    tail_ok = (per_point <= 1e-2) | inside
    return dict(n=n, within_1e4=int(within.sum()), frac_within=float(within.mean()),
                in_envelope=int((~within & inside).sum()), failures=int((~within & ~tail_ok).sum()),
                worst=float(per_point.max()), worst_index=int(per_point.argmax()))


def assert_bake_parity(gpu: np.ndarray, res: dict, min_frac: float = 0.999):
    r = bake_report(gpu, res)
    msg = (f"{r['within_1e4']}/{r['n']} points within 1e-4, {r['in_envelope']} in the tie "
           f"envelope, {r['failures']} failures, worst rel {r['worst']:.3e} at point {r['worst_index']}")
    assert r["frac_within"] >= min_frac and r["failures"] == 0, msg
    return r


def assert_close_rel(gpu, oracle, tol: float, floor: float = 1e-6, what: str = ""):
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(oracle, dtype=np.float64)
    tau = plane_tau(o.reshape(o.shape[0], -1), floor).reshape((o.shape[0],) + (1,) * (o.ndim - 1))
    rel = np.abs(g - o) / np.maximum(np.abs(o), tau)
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= tol, f"{what}: worst relative error {worst:.3e} > {tol:g} at {np.unravel_index(rel.argmax(), rel.shape)}"
    return worst
