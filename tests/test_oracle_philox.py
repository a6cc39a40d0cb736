"""Pins of the oracle's Gaussian sketch (Algorithm 2, step 1: Pi ~ N(0,1)).

The Philox words are pinned bit for bit by published known-answer vectors;
the Box-Muller normals by their distribution."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


def test_philox_known_answer_vectors(kat_vectors):
    assert len(kat_vectors) == 3
    for ctr, key, want in kat_vectors:
        got = philox.philox4x32_10(np.array(ctr, dtype=np.uint64), key)
        assert [int(x) for x in got] == want


def test_philox_vectorized_matches_scalar(kat_vectors):
    ctrs = np.array([c for c, _, _ in kat_vectors[:1]] * 3, dtype=np.uint64)
    got = philox.philox4x32_10(ctrs, kat_vectors[0][1])
    for row in got:
        assert [int(x) for x in row] == kat_vectors[0][2]


def test_counter_layout_uses_high_word():
    # pair index j >= 2^32 must set the second counter word
    w = philox.philox_words(7, 3)
    ctr = np.array([[2, 0, 0, 0]], dtype=np.uint64)
    assert np.array_equal(w[2], philox.philox4x32_10(ctr, (7, 0))[0])
    hi = philox.philox4x32_10(np.array([[0, 1, 0, 0]], dtype=np.uint64), (7, 0))[0]
    assert not np.array_equal(hi, w[0])


def test_gaussian_moments_and_ks():
    z = philox.gaussian(12345, 1000, 1000).ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 5.0 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two normals of one Box-Muller pair are uncorrelated
    pairs = z.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5.0 / np.sqrt(n / 2)


def test_gaussian_layout_and_determinism():
    a = philox.gaussian(3, 37, 11)
    b = philox.gaussian(3, 1, 37 * 11).reshape(37, 11)
    assert np.array_equal(a, b)                  # row-major element order
    assert np.array_equal(a, philox.gaussian(3, 37, 11))
    assert not np.allclose(a, philox.gaussian(4, 37, 11))
    odd = philox.gaussian(3, 1, 5)               # odd count drops the last normal
    assert np.array_equal(odd.ravel(), a.ravel()[:5])


@pytest.mark.parametrize("seed", [0, 2**32 + 5, 2**64 - 1])
def test_gaussian_finite_for_extreme_seeds(seed):
    z = philox.gaussian(seed, 64, 64)
    assert np.all(np.isfinite(z))
