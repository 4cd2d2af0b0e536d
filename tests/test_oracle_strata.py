"""Pins of the oracle's stratified lobe uniforms against facts other than
their own code: the Philox block they start from (itself pinned by the
generator's known-answer vectors), the geometry of Morton codes on the unit
square, and the closed-form integral of a smooth integrand together with the
variance plain Monte Carlo would have on it."""
import numpy as np
import pytest

from oracle import bake as ob

SEED = 0x0123456789ABCDEF


def _block(p, lobe, s):
    ctr = np.stack([p & 0xFFFFFFFF, p >> 32, lobe, s], axis=1).astype(np.uint64).astype(np.uint32)
    key = np.tile(np.array([SEED & 0xFFFFFFFF, SEED >> 32], np.uint64), (len(p), 1))
    return ob.philox(ctr, key.astype(np.uint32)).astype(np.uint64)


def _morton(col, row):
    """Morton code of a 2^16 x 2^16 grid cell: bit i of the column goes to
    bit 2i, bit i of the row to bit 2i + 1."""
    code = np.zeros(col.shape, np.uint64)
    for i in range(16):
        code |= ((col >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i)
        code |= ((row >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i + 1)
    return code


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 100, 128, 1000, 65536])
def test_sample_lies_in_its_segment_of_the_curve(n):
    """The top 16 bits of (xi1, xi2) name the cell whose Morton code is the
    sample's point U on the curve; U lies in the s-th of n segments of width
    floor(2^32 / n), offset by floor(u0 W / 2^32); the low 8 bits are the top
    bytes of u1 and u2."""
    rng = np.random.default_rng(n)
    m = 4096
    p = rng.integers(0, 1 << 40, size=m, dtype=np.int64)
    lobe = rng.integers(0, 17, size=m).astype(np.int64)
    s = rng.integers(0, n, size=m).astype(np.int64)
    xi1, xi2 = ob.lobe_uniforms(SEED, p, lobe, s, n)
    a1 = xi1 * 2.0 ** 24
    a2 = xi2 * 2.0 ** 24
    assert np.all(a1 == np.floor(a1)) and np.all(a2 == np.floor(a2))
    assert a1.min() >= 0 and a1.max() < 2 ** 24 and a2.min() >= 0 and a2.max() < 2 ** 24
    a1 = a1.astype(np.uint64)
    a2 = a2.astype(np.uint64)
    U = _morton(a1 >> np.uint64(8), a2 >> np.uint64(8))
    W = np.uint64((1 << 32) // n)
    np.testing.assert_array_equal(U // W, s.astype(np.uint64))
    u = _block(p, lobe, s)
    np.testing.assert_array_equal(U - s.astype(np.uint64) * W, (u[:, 0] * W) >> np.uint64(32))
    np.testing.assert_array_equal(a1 & np.uint64(255), u[:, 1] >> np.uint64(24))
    np.testing.assert_array_equal(a2 & np.uint64(255), u[:, 2] >> np.uint64(24))


@pytest.mark.parametrize("side", [2, 4, 16])
def test_power_of_four_counts_fill_the_dyadic_grid(side):
    """With n = side^2 samples (side a power of two), segment s of the Morton
    curve is one cell of the side x side grid: its column holds the even
    bits of s, its row the odd bits; so every cell gets exactly one sample."""
    n = side * side
    s = np.arange(n, dtype=np.int64)
    for p in (0, 12345, (1 << 33) + 7):
        xi1, xi2 = ob.lobe_uniforms(SEED, np.full(n, p), 2, s, n)
        col = np.floor(xi1 * side).astype(np.int64)
        row = np.floor(xi2 * side).astype(np.int64)
        want_col = sum(((s >> (2 * i)) & 1) << i for i in range(8))
        want_row = sum(((s >> (2 * i + 1)) & 1) << i for i in range(8))
        np.testing.assert_array_equal(col, want_col)
        np.testing.assert_array_equal(row, want_row)
        assert len(set(zip(col.tolist(), row.tolist()))) == n


@pytest.mark.parametrize("n,ratio", [(64, 0.25), (100, 0.35), (128, 0.2)])
def test_stratified_estimate_is_unbiased_and_tighter(n, ratio):
    """For f(x, y) = x^2 + x y + sin(pi y), whose integral over the unit
    square is 1/3 + 1/4 + 2/pi: the per-point estimates over n samples
    average to the integral within four standard errors, and their spread
    is well below the sqrt(Var f / n) of independent samples."""
    m = 3000
    p = np.repeat(np.arange(m, dtype=np.int64) + 77, n)
    s = np.tile(np.arange(n, dtype=np.int64), m)
    xi1, xi2 = ob.lobe_uniforms(SEED, p, 0, s, n)
    f = xi1 ** 2 + xi1 * xi2 + np.sin(np.pi * xi2)
    est = f.reshape(m, n).mean(axis=1)
    exact = 1.0 / 3.0 + 0.25 + 2.0 / np.pi
    # variance of f under independent uniform samples (midpoint rule, 2000^2)
    g = (np.arange(2000) + 0.5) / 2000
    X, Y = np.meshgrid(g, g, indexing="ij")
    F = X ** 2 + X * Y + np.sin(np.pi * Y)
    plain = np.sqrt((np.mean(F ** 2) - np.mean(F) ** 2) / n)
    spread = est.std()
    assert spread < ratio * plain
    assert abs(est.mean() - exact) < 4.0 * spread / np.sqrt(m) + 1e-7
