"""Pins of the oracle's stratified lobe uniforms against facts other than
their own code: the Philox block they start from (itself pinned by the
generator's known-answer vectors), the geometry of a Hilbert curve on a 4 x 4
grid and of Morton codes inside its cells, and the closed-form integral of a
smooth integrand together with the variance plain Monte Carlo would have on
it."""
import numpy as np
import pytest

from oracle import bake as ob

SEED = 0x0123456789ABCDEF


def _block(p, lobe, s):
    ctr = np.stack([p & 0xFFFFFFFF, p >> 32, lobe, s], axis=1).astype(np.uint64).astype(np.uint32)
    key = np.tile(np.array([SEED & 0xFFFFFFFF, SEED >> 32], np.uint64), (len(p), 1))
    return ob.philox(ctr, key.astype(np.uint32)).astype(np.uint64)


def _morton(col, row, bits=16):
    """Morton code of a cell: bit i of the column goes to bit 2i, bit i of
    the row to bit 2i + 1."""
    code = np.zeros(col.shape, np.uint64)
    for i in range(bits):
        code |= ((col >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i)
        code |= ((row >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i + 1)
    return code


def _top_cells():
    """Cells of the 4 x 4 grid holding samples 0..15 of 16."""
    xi1, xi2 = ob.lobe_uniforms(SEED, np.full(16, 5), 1, np.arange(16), 16)
    return list(zip(np.floor(xi1 * 4).astype(int).tolist(), np.floor(xi2 * 4).astype(int).tolist()))


def test_top_level_is_a_hilbert_curve():
    """The 16 segments of the curve visit the cells of the 4 x 4 grid once
    each, every step to an edge neighbour, from (0, 0) to (3, 0), finishing
    each 2 x 2 quadrant before the next, the quadrants in the order
    (0, 0), (0, 1), (1, 1), (1, 0) -- a Hilbert curve (consecutive segments
    are never far apart in the square, unlike a Morton order's jumps)."""
    cells = _top_cells()
    assert len(set(cells)) == 16
    assert cells[0] == (0, 0) and cells[-1] == (3, 0)
    for (x0, y0), (x1, y1) in zip(cells, cells[1:]):
        assert abs(x0 - x1) + abs(y0 - y1) == 1
    quads = [(x // 2, y // 2) for x, y in cells]
    assert quads == [q for q in [(0, 0), (0, 1), (1, 1), (1, 0)] for _ in range(4)]
    # with 4 samples each quadrant holds one, in the same order
    xi1, xi2 = ob.lobe_uniforms(SEED, np.full(4, 9), 0, np.arange(4), 4)
    got = list(zip((xi1 >= 0.5).astype(int).tolist(), (xi2 >= 0.5).astype(int).tolist()))
    assert got == [(0, 0), (0, 1), (1, 1), (1, 0)]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 100, 128, 1000, 65536])
def test_sample_lies_in_its_segment_of_the_curve(n):
    """The point U on the 32-bit line, rebuilt from (xi1, xi2) -- the top
    cell's position along the curve, then the Morton code of the point
    inside it -- lies in the s-th of n segments of width floor(2^32 / n),
    offset by floor(u0 W / 2^32); the low 8 bits of each uniform are the top
    bytes of u1 and u2."""
    order = {c: d for d, c in enumerate(_top_cells())}
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
    X, Y = a1 >> np.uint64(8), a2 >> np.uint64(8)
    d = np.array([order[(int(x), int(y))] for x, y in zip(X >> np.uint64(14), Y >> np.uint64(14))],
                 dtype=np.uint64)
    low = _morton(X & np.uint64(0x3FFF), Y & np.uint64(0x3FFF), bits=14)
    U = (d << np.uint64(28)) | low
    W = np.uint64((1 << 32) // n)
    np.testing.assert_array_equal(U // W, s.astype(np.uint64))
    u = _block(p, lobe, s)
    np.testing.assert_array_equal(U - s.astype(np.uint64) * W, (u[:, 0] * W) >> np.uint64(32))
    np.testing.assert_array_equal(a1 & np.uint64(255), u[:, 1] >> np.uint64(24))
    np.testing.assert_array_equal(a2 & np.uint64(255), u[:, 2] >> np.uint64(24))


@pytest.mark.parametrize("side", [8, 16])
def test_power_of_four_counts_fill_the_dyadic_grid(side):
    """With n = side^2 samples, each cell of the side x side grid gets
    exactly one; the samples come in runs of n/16 per cell of the 4 x 4
    grid, in the curve's order, and inside such a cell sample s sits at the
    column of the even bits of s mod n/16 and the row of its odd bits."""
    n = side * side
    sub = side // 4
    top = _top_cells()
    s = np.arange(n, dtype=np.int64)
    for p in (0, 12345, (1 << 33) + 7):
        xi1, xi2 = ob.lobe_uniforms(SEED, np.full(n, p), 2, s, n)
        col = np.floor(xi1 * side).astype(np.int64)
        row = np.floor(xi2 * side).astype(np.int64)
        assert len(set(zip(col.tolist(), row.tolist()))) == n
        r = s % (n // 16)
        want_col = np.array([top[k][0] for k in s // (n // 16)]) * sub + \
            sum(((r >> (2 * i)) & 1) << i for i in range(8))
        want_row = np.array([top[k][1] for k in s // (n // 16)]) * sub + \
            sum(((r >> (2 * i + 1)) & 1) << i for i in range(8))
        np.testing.assert_array_equal(col, want_col)
        np.testing.assert_array_equal(row, want_row)


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
