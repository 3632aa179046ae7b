"""Pins of the oracle's Legendre basis and random-subset sampler against closed forms,
quadrature identities, published generator outputs and exhaustive enumeration."""
import itertools

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.basis import legendre_P, legendre_orthonormal, to_reference
from oracle.sampler import (GAMMA, bounded, sample_without_replacement, splitmix64,
                            stream_state)


def test_legendre_closed_forms():
    t = np.linspace(-1, 1, 37)
    P = legendre_P(t, 3)
    np.testing.assert_allclose(P[:, 0], 1.0, rtol=0, atol=0)
    np.testing.assert_allclose(P[:, 1], t, rtol=0, atol=0)
    np.testing.assert_allclose(P[:, 2], 0.5 * (3 * t * t - 1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(P[:, 3], 0.5 * (5 * t ** 3 - 3 * t), rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 5, 15, 31, 40])
def test_legendre_endpoints(p):
    P = legendre_P(np.array([-1.0, 1.0]), p)
    n = np.arange(p + 1)
    np.testing.assert_allclose(P[1], 1.0, atol=1e-13)
    np.testing.assert_allclose(P[0], (-1.0) ** n, atol=1e-13)


@pytest.mark.parametrize("p", [3, 15, 31])
def test_legendre_orthonormal_under_gauss_quadrature(p):
    # Gauss-Legendre with nq nodes is exact for degree <= 2 nq - 1; phi_a phi_b has degree <= 2p.
    nq = p + 1
    x, w = npleg.leggauss(nq)
    Phi = legendre_orthonormal(x, p)
    M = 0.5 * (Phi * w[:, None]).T @ Phi
    np.testing.assert_allclose(M, np.eye(p + 1), atol=1e-12)


def test_legendre_matches_numpy_legval():
    t = np.random.default_rng(0).uniform(-1, 1, 101)
    P = legendre_P(t, 20)
    for m in range(21):
        c = np.zeros(m + 1)
        c[m] = 1.0
        np.testing.assert_allclose(P[:, m], npleg.legval(t, c), rtol=1e-12, atol=1e-13)


def test_reference_map():
    assert to_reference(0.0, 0.0, 4.0) == -1.0
    assert to_reference(4.0, 0.0, 4.0) == 1.0
    assert to_reference(2.0, 0.0, 4.0) == 0.0


def test_splitmix64_published_outputs():
    # Reference outputs of SplitMix64 (Vigna's splitmix64.c): state 0 -> first output
    # 0xE220A8397B1DCDAF; state 1234567 -> the five values below.
    assert int(splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF
    assert [int(v) for v in splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_splitmix64_counter_form():
    # The i-th output depends only on state + (i+1) * gamma: restarting there gives it back.
    z = splitmix64(99, 10)
    for i in range(10):
        s = (99 + i * GAMMA) % (1 << 64)
        assert int(splitmix64(s, 1)[0]) == int(z[i])


def test_bounded_matches_bigint():
    rng = np.random.default_rng(3)
    r = rng.integers(0, 2 ** 63, size=1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    n = rng.integers(1, 2 ** 32 - 1, size=1000, dtype=np.uint64)
    got = bounded(r, n)
    exp = [(int(a) * int(b)) >> 64 for a, b in zip(r, n)]
    assert [int(g) for g in got] == exp


def test_sample_distinct_sorted_and_edge_sizes():
    s = sample_without_replacement(7, 2, 1000, 300)
    assert len(s) == 300 and len(np.unique(s)) == 300 and np.all(np.diff(s) > 0)
    assert s.min() >= 0 and s.max() < 1000
    np.testing.assert_array_equal(sample_without_replacement(7, 2, 50, 50), np.arange(50))
    assert sample_without_replacement(7, 2, 50, 0).size == 0
    with pytest.raises(ValueError):
        sample_without_replacement(7, 2, 5, 6)


def test_sample_uniform_over_subsets():
    # Exhaustive: every 2-subset of 5 items must be (nearly) equally likely over many seeds.
    counts = {c: 0 for c in itertools.combinations(range(5), 2)}
    trials = 20000
    for seed in range(trials):
        counts[tuple(int(v) for v in sample_without_replacement(seed, 2, 5, 2))] += 1
    exp = trials / len(counts)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 30.0      # 9 degrees of freedom; p ~ 4e-4 at 30


def test_stream_seeds_differ():
    a = sample_without_replacement(1, 1, 10000, 100)
    b = sample_without_replacement(1, 2, 10000, 100)
    assert not np.array_equal(a, b)
    assert stream_state(3, 2) == 3 * 256 + 2
