"""Pin of the oracle's KL mode order (Sec. 3.3: the input basis is the
leading Karhunen-Loeve modes of the field, i.e. those of largest amplitude).

The field of the workload is m = sum a_k xi_k s_k(x) with sine modes s_k
and amplitudes a_k = (pi^2 |k|^2 + 25)^(-e) (e = 1.25 on the square, 1.5 on
the cube).  The leading r_m modes are the r_m largest a_k; where the cut
falls inside a group of equal amplitudes, the lexicographically smallest
multi-indices are taken.  These tests rank the modes by the amplitude
itself, computed here from that formula, so an ordering by increasing
amplitude, by j + k, or without the lexicographic tie-break fails.
"""
import itertools
import math

import pytest

from oracle import surrogate


def _amplitude(idx, expo):
    return (math.pi ** 2 * sum(v * v for v in idx) + 25.0) ** (-expo)


def _leading_by_amplitude(K1, dim, expo, r):
    modes = list(itertools.product(range(1, K1 + 1), repeat=dim))
    # decreasing amplitude; equal amplitudes in lexicographic order
    modes.sort(key=lambda t: (-_amplitude(t, expo), t))
    return modes[:r]


@pytest.mark.parametrize("K1,dim,expo,r_m,tie", [(16, 2, 1.25, 100, 145), (10, 3, 1.5, 200, 65),
                                                 (8, 2, 1.25, 64, None), (16, 2, 1.25, 256, None)])
def test_kl_order_is_decreasing_amplitude_with_lexicographic_ties(K1, dim, expo, r_m, tie):
    order = surrogate.kl_order(K1, dim)
    assert len(order) == K1 ** dim and len(set(order)) == K1 ** dim
    amps = [_amplitude(t, expo) for t in order]
    for a, b, ta, tb in zip(amps, amps[1:], order, order[1:]):
        assert a >= b                                 # non-increasing amplitude
        if a == b:
            assert ta < tb                            # ties: lexicographic ascending
    assert order[:r_m] == _leading_by_amplitude(K1, dim, expo, r_m)
    if tie is not None:
        # the cut falls strictly inside a group of equal |k|^2, so the
        # tie-break decides which members are kept
        sq = [sum(v * v for v in t) for t in order]
        assert sq[r_m - 1] == tie and sq[r_m] == tie
        group = [t for t in order if sum(v * v for v in t) == tie]
        kept = [t for t in order[:r_m] if sum(v * v for v in t) == tie]
        assert 0 < len(kept) < len(group) and kept == sorted(group)[:len(kept)]


def test_encode_takes_the_leading_coordinates():
    """encode() returns the xi of the leading modes in that order."""
    import numpy as np
    K1 = 16
    rng = np.random.default_rng(7)
    xi = rng.standard_normal((3, K1, K1))
    enc = surrogate.encode(xi, 100)
    lead = _leading_by_amplitude(K1, 2, 1.25, 100)
    expect = np.stack([xi[:, j - 1, k - 1] for (j, k) in lead], axis=1)
    assert np.array_equal(enc, expect)
    xi3 = rng.standard_normal((2, 10, 10, 10))
    enc3 = surrogate.encode(xi3, 200)
    lead3 = _leading_by_amplitude(10, 3, 1.5, 200)
    assert np.array_equal(enc3, np.stack([xi3[:, a - 1, b - 1, c - 1] for (a, b, c) in lead3], axis=1))
