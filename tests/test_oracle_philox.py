"""Pins of the oracle's Philox4x32-10 against things other than itself:
the generator's published known-answer vectors, rocRAND's independent
open-source engine run on the host, and uniformity of the derived floats."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import bake as ob

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append(v)
    return np.array(rows, dtype=np.uint64).astype(np.uint32)


def test_known_answer_vectors():
    kat = _kat()
    out = ob.philox(kat[:, 0:4], kat[:, 4:6])
    np.testing.assert_array_equal(out, kat[:, 6:10])


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc for the host build of rocRAND's engine")
def test_matches_rocrand_engine():
    """rocRAND's philox4x32_10_engine(seed, subsequence, offset) evaluates the
    block with key = seed, counter = (offset/4 lo, hi, subsequence lo, hi)."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "probe")
        subprocess.run(["hipcc", "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand.cpp")],
                       check=True, capture_output=True, cwd=d)
        rng = np.random.default_rng(11)
        rec = rng.integers(0, 2 ** 32, size=(200000, 6), dtype=np.uint64).astype(np.uint32)
        rec[:, 1] &= 0x3FFFFFFF   # offset * 4 must fit the engine's 64-bit offset
        rec[:64, 0:4] = 0
        rec[:64, 2] = np.arange(64)
        inp, outp = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        rec.tofile(inp)
        subprocess.run([exe, inp, outp], check=True)
        ref = np.fromfile(outp, dtype=np.uint32).reshape(-1, 4)
    np.testing.assert_array_equal(ob.philox(rec[:, 0:4], rec[:, 4:6]), ref)


def test_uniform_24bit_floats_chi2():
    """xi = (u >> 8) * 2^-24 over 2^20 consecutive sample counters is
    uniform on [0, 1): chi-square over 256 bins below the 0.999 quantile."""
    from scipy import stats
    n = 1 << 20
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n) // 64
    ctr[:, 3] = np.arange(n) % 64
    key = np.tile(np.array([2001, 0], np.uint32), (n, 1))
    u = ob.philox(ctr, key)
    for col in (0, 1):
        xi = (u[:, col] >> 8).astype(np.float64) / 2 ** 24
        assert xi.min() >= 0.0 and xi.max() < 1.0
        h, _ = np.histogram(xi, bins=256, range=(0, 1))
        chi2 = ((h - n / 256) ** 2 / (n / 256)).sum()
        assert chi2 < stats.chi2.ppf(0.999, 255)
    # the two streams are uncorrelated
    x0 = (u[:, 0] >> 8) / 2.0 ** 24
    x1 = (u[:, 1] >> 8) / 2.0 ** 24
    assert abs(np.corrcoef(x0, x1)[0, 1]) < 5.0 / np.sqrt(n)
