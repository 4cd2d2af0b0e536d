"""Mutation sweep of the oracle: each entry plants one plausible mistake (a
dropped term, a wrong sign, power, index or operand) in a temporary copy of
``oracle/``; the oracle's pins (every ``tests/test_oracle_*.py``) must then
fail.  A control copy without a mutation must pass, so a failure is the
pins' doing and not the harness's.

The mistakes are planted on the CPU, in the oracle only; nothing here
touches the GPU library.  Marked slow: one pytest run of the pins per
mutant, several in parallel.
"""
import ast
import os
import re
import shutil
import signal
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C = "oracle/fipt_oracle.c"
# (name, file, [(old, new, which occurrence or None for the only one)]
#  [, pin files to run first])
MUTANTS = [
    # microfacet model and the estimator of Eq. 6 / 7
    ("alpha = sigma instead of sigma^2", C,
     [("double alpha = sigma[k] * sigma[k];", "double alpha = sigma[k];", 0)]),
    ("one Smith G1 dropped", C,
     [("        G = orc_ggx_G1(alpha, ci) * orc_ggx_G1(alpha, cos_o);",
       "        G = orc_ggx_G1(alpha, cos_o);", None)]),
    ("Schlick power 4 instead of 5", C,
     [("*F1 = one_minus * one_minus * one_minus * one_minus * one_minus;",
       "*F1 = one_minus * one_minus * one_minus * one_minus;", None)]),
    ("F0 and F1 terms swapped", C,
     [("int j0 = 3 + 3 * k, j1 = 3 + 3 * K + 3 * k;", "int j1 = 3 + 3 * k, j0 = 3 + 3 * K + 3 * k;", 0)]),
    ("n.m missing from the sample weight", C,
     [("return G * om / (cos_o * cm);", "return G * om / cos_o;", None)]),
    ("GGX D with the denominator not squared", C,
     [("double d = c2 * c2 * (a2 + tan2) * (a2 + tan2);", "double d = c2 * c2 * (a2 + tan2);", None)]),
    ("G1 with alpha instead of alpha^2", C,
     [("return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));",
       "return 2.0 / (1.0 + sqrt(1.0 + alpha * tan2));", None)]),
    ("GGX sampler with alpha instead of alpha^2", C,
     [("double tan2 = alpha * alpha * xi1 / (1.0 - xi1);", "double tan2 = alpha * xi1 / (1.0 - xi1);", None)]),
    ("reflection without the factor 2", C,
     [("for (int k = 0; k < 3; ++k) wi[k] = 2.0 * om * m[k] - wo[k];",
       "for (int k = 0; k < 3; ++k) wi[k] = om * m[k] - wo[k];", 0)]),
    # (dropping only the wi test is no mistake: G1 is zero below the horizon)
    ("no horizon rejection: wi test and G1's guard dropped", C,
     [("        if (ci <= 0.0) return 0.0;\n        /* wi.m", "        /* wi.m", None),
      ("    if (cos_v <= 0.0) return 0.0;\n    double c2 = cos_v * cos_v;",
       "    double c2 = cos_v * cos_v;", None)]),
    ("cosine sampler: cos theta = sqrt(xi1)", C,
     [("out[2] = sqrt(1.0 - xi1);", "out[2] = sqrt(xi1);", None)]),
    ("frame: sign error in t", C,
     [("t[2] = -s * n[0];", "t[2] = s * n[0];", None)]),
    ("mean divides by spp + 1", C,
     [("double cnt = (k < 3) ? (double)spp_d : (double)spp_s;\n                out[k * n_idx + q]",
       "double cnt = (k < 3) ? (double)spp_d : (double)(spp_s + 1);\n                out[k * n_idx + q]", 0)]),
    # random numbers
    ("Philox Weyl constant off by two", C,
     [("k0 += 0x9E3779B9u;", "k0 += 0x9E3779B7u;", None)]),
    ("xi2's low bits from the wrong Philox word", C,
     [("(double)(u[2] >> 24)) / 16777216.0;", "(double)(u[1] >> 24)) / 16777216.0;", None)]),
    ("Morton code: y from the even bits", C,
     [("Y |= (uint32_t)((U >> (2 * i + 1)) & 1u) << i;", "Y |= (uint32_t)((U >> (2 * i)) & 1u) << i;", None)]),
    # ray casting and the radiance query of Eq. 9
    ("ray origin offset against the normal", C,
     [("for (int k = 0; k < 3; ++k) o[k] = x[k] + eps * n[k];",
       "for (int k = 0; k < 3; ++k) o[k] = x[k] - eps * n[k];", 0)]),
    ("farthest hit instead of nearest", C,
     [("    out->nominal.t = INFINITY;", "    out->nominal.t = -INFINITY;", None),
      ("(t < out->nominal.t || (t == out->nominal.t && f < out->nominal.tri))",
       "(t > out->nominal.t || (t == out->nominal.t && f < out->nominal.tri))", None)]),
    ("distance ties to the higher triangle index", C,
     [("(t == out->nominal.t && f < out->nominal.tri)", "(t == out->nominal.t && f > out->nominal.tri)", None)]),
    ("shared-edge fallback removed", C,
     [("if (out->nominal.tri < 0 && fallback.tri >= 0) {", "if (0) {", None)]),
    ("barycentric weights of vertices 1 and 2 swapped", C,
     [("double w1 = h->b1, w2 = h->b2, w0 = 1.0 - w1 - w2;", "double w1 = h->b2, w2 = h->b1, w0 = 1.0 - w1 - w2;", None)]),
    ("cache and emission combined by max instead of sum", C,
     [("for (int c = 0; c < 3; ++c) R[c] += S->cache[c * S->T + f];",
       "for (int c = 0; c < 3; ++c) R[c] = fmax(R[c], S->cache[c * S->T + f]);", None)]),
    ("emission dropped from the radiance", C,
     [("for (int c = 0; c < 3; ++c) R[c] = S->emission[c * S->T + f];",
       "for (int c = 0; c < 3; ++c) R[c] = 0.0;", None)]),
    ("camera aspect inverted", C,
     [("double aspect = (double)W / (double)H;", "double aspect = (double)H / (double)W;", None)]),
    # stage-3 refinement (Eq. 10 / 11): pins in test_oracle_refine.py first
    ("refine: MIS weight of a BRDF-sampled emitter hit inverted", C,
     [("w = pb_prev / (pb_prev + pl);", "w = pl / (pb_prev + pl);", None)], ["test_oracle_refine.py"]),
    ("refine: emitter sample density without the emitter's cosine", C,
     [("double pl = dist * dist / (cz * M->n_emit * area);",
       "double pl = dist * dist / (M->n_emit * area);", None)], ["test_oracle_refine.py"]),
    ("refine: mixture density counts the GGX half twice", C,
     [("return 0.5 * ps + 0.5 * ci / ORC_PI;", "return ps + 0.5 * ci / ORC_PI;", None)],
     ["test_oracle_refine.py"]),
    ("refine: path throughput not divided by the density", C,
     [("for (int c = 0; c < 3; ++c) T[c] *= fv[c] / pb;", "for (int c = 0; c < 3; ++c) T[c] *= fv[c];", None)],
     ["test_oracle_refine.py"]),
    ("refine: diffuse BRDF without 1/pi", C,
     [("out[c] = kd / ORC_PI * ci + (ks * (1.0 - F1) + F1) * spec_base;",
       "out[c] = kd * ci + (ks * (1.0 - F1) + F1) * spec_base;", None)], ["test_oracle_refine.py"]),
    ("refine: Fresnel split without ks", C,
     [("out[c] = kd / ORC_PI * ci + (ks * (1.0 - F1) + F1) * spec_base;",
       "out[c] = kd / ORC_PI * ci + spec_base;", None)], ["test_oracle_refine.py"]),
    ("refine: sigma threshold reversed", C,
     [("int diffuse = mat[3] > M->sigma_diffuse;", "int diffuse = mat[3] < M->sigma_diffuse;", None)],
     ["test_oracle_refine.py"]),
    ("refine: points on emitters not uniform in area", C,
     [("double su = sqrt(unif24(u[1])), b1", "double su = unif24(u[1]), b1", None)],
     ["test_oracle_refine.py"]),
    ("refine: material grid x and y swapped", C,
     [("int64_t node = (i0[0] + dx) + R * ((i0[1] + dy) + R * (int64_t)(i0[2] + dz));",
       "int64_t node = (i0[1] + dy) + R * ((i0[0] + dx) + R * (int64_t)(i0[2] + dz));", None)],
     ["test_oracle_refine.py"]),
    # factored render, loss and gradient (Eq. 5, 8, 2)
    ("specular base reflectance 0.4 instead of 0.04", "oracle/render.py",
     [("ks = 0.04 * (1.0 - m) + a * m", "ks = 0.4 * (1.0 - m) + a * m", None)]),
    ("lerp weights swapped", "oracle/render.py",
     [("L0 = (1.0 - t) * S0j + t * S0k", "L0 = t * S0j + (1.0 - t) * S0k", None)]),
    ("metallic gradient with the wrong sign on Ld", "oracle/render.py",
     [("grad[4] = np.sum(g * (-r[\"a\"] * r[\"Ld\"] + (r[\"a\"] - 0.04) * r[\"L0\"]), axis=0)\n    dsig",
       "grad[4] = np.sum(g * (r[\"a\"] * r[\"Ld\"] + (r[\"a\"] - 0.04) * r[\"L0\"]), axis=0)\n    dsig", 0)]),
    ("roughness gradient not divided by the level gap", "oracle/render.py",
     [("dsig = np.sum(g * (r[\"ks\"] * r[\"dS0\"] + r[\"dS1\"]), axis=0) / r[\"dsig\"]\n    grad[3] = np.where(r[\"clamped\"], 0.0, dsig)\n    return loss",
       "dsig = np.sum(g * (r[\"ks\"] * r[\"dS0\"] + r[\"dS1\"]), axis=0)\n    grad[3] = np.where(r[\"clamped\"], 0.0, dsig)\n    return loss", None)]),
    ("bracket at the left-hand segment of a knot", "oracle/render.py",
     [("j = np.searchsorted(g, s, side=\"right\") - 1", "j = np.searchsorted(g, s, side=\"left\") - 1", None)]),
    ("mask scales the loss by (1 - alpha) only once in the gradient", "oracle/render.py",
     [("g = gh * (1.0 - al)                                          # dl/dLr",
       "g = gh                                                       # dl/dLr", None)]),
    # other next-row oracles
    ("median: upper middle value for even counts", "oracle/emission.py",
     [("out[c, t] = vals[(k - 1) // 2]", "out[c, t] = vals[k // 2]", None)]),
    ("voxel pooling: sum instead of mean", "oracle/cache.py",
     [("cache[:, seen] = sums[:, seen] / counts[seen]", "cache[:, seen] = sums[:, seen]", None)]),
    ("hash prime of y replaced", "oracle/hashgrid.py",
     [("PRIMES = (1, 2654435761, 805459861)", "PRIMES = (1, 2654435769, 805459861)", None)]),
    ("trilinear grid: clamp removed", "oracle/render.py",
     [("    u = np.clip(u, 0.0, res - 1)\n", "", None)]),
]

COPY_DIRS = ("oracle", "synth")
# the pin files (this sweep itself excluded: a copy must not run it again)
ORACLE_TESTS = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                      if re.fullmatch(r"test_oracle_[a-z]+\.py", f) and f != os.path.basename(__file__))
# Pin files run first for a mutant of each oracle file (every other pin
# file still runs after them until one fails): only the order changes, so
# a caught mutant stops early.
FIRST = {
    C: ["test_oracle_microfacet.py", "test_oracle_philox.py", "test_oracle_strata.py",
        "test_oracle_raycast.py", "test_oracle_primary.py", "test_oracle_bake.py"],
    "oracle/render.py": ["test_oracle_render.py", "test_oracle_masked.py"],
    "oracle/emission.py": ["test_oracle_emission.py"],
    "oracle/cache.py": ["test_oracle_cache.py"],
    "oracle/hashgrid.py": ["test_oracle_hashgrid.py"],
}


def _workspace(tmp: str) -> str:
    """A copy of what the oracle's pins load: oracle/ (sources only, so the
    C file is rebuilt), synth/, the pin files, conftest, golden data."""
    dst = os.path.join(tmp, "repo")
    ignore = shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__")
    for d in COPY_DIRS:
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d), ignore=ignore)
    os.makedirs(os.path.join(dst, "tests"))
    for f in ORACLE_TESTS + ["conftest.py", "philox_rocrand.cpp"]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)
    return dst


def _apply(repo: str, path: str, edits) -> None:
    full = os.path.join(repo, path)
    src = open(full).read()
    for old, new, which in edits:
        count = src.count(old)
        if which is None:
            assert count == 1, f"{path}: {old!r} occurs {count} times"
            src = src.replace(old, new)
        else:
            assert count > which, f"{path}: {old!r} occurs {count} times"
            at = -1
            for _ in range(which + 1):
                at = src.index(old, at + 1)
            src = src[:at] + new + src[at + len(old):]
    open(full, "w").write(src)
    if path.endswith(".py"):
        ast.parse(src)
    else:
        # the mutant must still compile, so a failing run is the pins' doing
        r = subprocess.run(["gcc", "-fsyntax-only", "-fopenmp", "-Wall", full],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def _run_pins(name, path, edits, first=None, threads: int = 2, limit_s: int = 300):
    with tempfile.TemporaryDirectory(prefix="orc_mut_") as tmp:
        repo = _workspace(tmp)
        if path:
            _apply(repo, path, edits)
        first = (first or []) + [f for f in FIRST.get(path, []) if f not in (first or [])]
        order = first + [f for f in ORACLE_TESTS if f not in first]
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), PYTHONDONTWRITEBYTECODE="1")
        env.pop("PYTHONPATH", None)
        # own session, so a run past its limit is ended with everything it started
        p = subprocess.Popen([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                              "-p", "no:cacheprovider"] + [f"tests/{f}" for f in order],
                             cwd=repo, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                             text=True, start_new_session=True)
        try:
            out, _ = p.communicate(timeout=limit_s)
        except subprocess.TimeoutExpired:
            os.killpg(p.pid, signal.SIGKILL)
            out, _ = p.communicate()
            return name, "timeout", out[-2000:]
        return name, p.returncode, out[-2000:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    jobs = [("control", None, None)] + MUTANTS
    with ThreadPoolExecutor(max_workers=4) as ex:
        # the control runs every pin; mutants stop at the first failing one
        results = list(ex.map(lambda m: _run_pins(*m), jobs))
    control = results[0]
    assert control[1] == 0, f"the unmutated copy must pass its pins:\n{control[2]}"
    survivors = []
    for name, rc, out in results[1:]:
        # exit code 1 = some test failed; a collection error or crash would
        # be another code and counts as a harness problem, not a catch
        if rc != 1 or " failed" not in out:   # "timeout" included
            survivors.append(f"{name} (exit {rc}): {out[-400:]}")
    assert not survivors, "mutants not caught by any pin:\n" + "\n".join(survivors)
