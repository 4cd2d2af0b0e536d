"""Pins of the oracle's per-triangle emission estimate (Eq. 13 with f = 0)
against facts other than its own code: numpy's median where the count is
odd, hand-worked small cases (even counts take the lower middle value), the
robustness that defines a median, and the recovery of the true emission
from noisy observations of emitters that reflect nothing."""
import numpy as np

from oracle import emission as oe


def test_odd_counts_match_numpy_median():
    rng = np.random.default_rng(1)
    T = 50
    tri = rng.integers(-1, T, size=20001)
    obs = rng.standard_normal((3, len(tri))).astype(np.float32) * 5
    emitter = np.ones(T, bool)
    got = oe.emission_median(tri, obs, T, emitter)
    for t in range(T):
        pix = tri == t
        if pix.sum() % 2 == 1:
            np.testing.assert_array_equal(got[:, t], np.median(obs[:, pix], axis=1).astype(np.float32))


def test_hand_cases():
    tri = np.array([0, 0, 0, 1, 1, 2, 1, 1, -1, 3])
    obs = np.array([[3.0, 1.0, 2.0, 10.0, 40.0, 7.0, 20.0, 30.0, 99.0, 5.0],
                    [0.0, 0.0, 0.0, -1.0, -4.0, 0.5, -2.0, -3.0, 99.0, 6.0],
                    [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 99.0, 7.0]], np.float32)
    emitter = np.array([True, True, True, False, True])
    got = oe.emission_median(tri, obs, 5, emitter)
    np.testing.assert_array_equal(got[:, 0], [2.0, 0.0, 1.0])      # three pixels: the middle one
    np.testing.assert_array_equal(got[:, 1], [20.0, -3.0, 1.0])    # four: the lower middle
    np.testing.assert_array_equal(got[:, 2], [7.0, 0.5, 1.0])      # one pixel: its value
    np.testing.assert_array_equal(got[:, 3], [0.0, 0.0, 0.0])      # not an emitter
    np.testing.assert_array_equal(got[:, 4], [0.0, 0.0, 0.0])      # an emitter no pixel sees


def test_outliers_do_not_move_it():
    """Replacing the values above (or below) the median by anything still
    above (below) it leaves the median unchanged."""
    rng = np.random.default_rng(2)
    n = 1001
    tri = np.zeros(n, int)
    obs = rng.uniform(0, 1, (3, n)).astype(np.float32)
    base = oe.emission_median(tri, obs, 1, [True])
    wild = obs.copy()
    for c in range(3):
        hi = wild[c] > base[c, 0]
        lo = wild[c] < base[c, 0]
        wild[c, hi] = 1e6
        wild[c, lo] = -1e6
    np.testing.assert_array_equal(oe.emission_median(tri, wild, 1, [True]), base)


def test_recovers_emission_from_noisy_observations():
    """Pixels of an emitter that reflects nothing observe its emission with
    1 % multiplicative noise: the estimate is within a few tenths of a
    percent, and non-emitters get zero."""
    rng = np.random.default_rng(3)
    T = 40
    Le = np.zeros((3, T), np.float32)
    em = rng.uniform(size=T) < 0.5
    Le[:, em] = rng.uniform(1, 50, size=em.sum())
    tri = rng.integers(0, T, size=200000)
    obs = (Le[:, tri] * (1 + 0.01 * rng.standard_normal((3, len(tri))))).astype(np.float32)
    got = oe.emission_median(tri, obs, T, em)
    np.testing.assert_allclose(got[:, em], Le[:, em], rtol=3e-3)
    assert (got[:, ~em] == 0).all()
