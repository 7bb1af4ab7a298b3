"""Pins of the oracle's random streams and acceptance tables.

* Philox4x32-10: against rocRAND's open-source engine (an independent
  implementation, compiled here as host code), through both its raw rounds
  and its public seed/subsequence/offset interface.
* splitmix64: only its Weyl-sequence structure, which holds for any
  finaliser.  The finaliser itself is "parity unpinned" (no published
  known-answer output is available here); it decides which stand-in instance
  a seed draws, and the generator pins check every drawn instance's validity.
* Threshold tables: against exp(-beta dE) 2^32 evaluated in 60-digit decimal
  arithmetic (Python's decimal module), which fixes the Metropolis
  acceptance min(1, exp(-beta dE)) of the Boltzmann law (App. A).
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

import oracle


def test_philox_matches_rocrand_rounds(rocrand_philox):
    rng = np.random.default_rng(2025)
    n = 40000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:100] = 0
    ctr[100:200] = 0xFFFFFFFF
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (0x12345678, 0x9ABCDEF0),
                (int(rng.integers(2 ** 32)), int(rng.integers(2 ** 32)))]:
        ref = np.zeros((n, 4), np.uint32)
        rocrand_philox.rocrand_philox_blocks(np.ascontiguousarray(ctr), key[0], key[1], ref, n)
        for i in range(0, n, 97):
            np.testing.assert_array_equal(oracle.philox(ctr[i], *key), ref[i])


def test_philox_matches_rocrand_public_engine(rocrand_philox):
    # seed -> key (lo, hi); subsequence -> counter words 2-3; offset/4 ->
    # counter words 0-1 (words 1 < 2^30 so the offset fits in 64 bits)
    rng = np.random.default_rng(7)
    n = 3000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 30) - 1
    seed = 0x0123456789ABCDEF
    ref = np.zeros((n, 4), np.uint32)
    rocrand_philox.rocrand_philox_public(seed, np.ascontiguousarray(ctr), ref, n)
    for i in range(n):
        np.testing.assert_array_equal(oracle.philox(ctr[i], seed & 0xFFFFFFFF, seed >> 32), ref[i])


def test_philox_words_are_uniform():
    # chi-squared over the top byte of 4 x 20000 words of consecutive counters
    words = np.concatenate([oracle.philox([i, 5, 6, 7], 11, 13) for i in range(20000)])
    hist = np.bincount(words >> 24, minlength=256)
    p = stats.chisquare(hist).pvalue
    assert p > 1e-4


def test_metropolis_and_init_streams_do_not_share_counters():
    # the init stream uses counter word 1 = 0xFFFFFFFF, which no Metropolis
    # counter (2s + c with s < 2^31 - 1) reaches; spot-check the mapping
    L = 8
    u = oracle.metropolis_uniform(L, 99, 4, 2, 0, 0)
    out = oracle.philox([0, 0, 2, 4], 99, 0)
    assert u == out[0]
    # site (x,y,z) = (3,5,6): colour 0, column floor(3/2) + 4*5 = 21,
    # call 21*2 + 1 = 43, word 6 % 4 = 2
    i = 3 + 8 * (5 + 8 * 6)
    u = oracle.metropolis_uniform(L, 99, 4, 2, 7, i)
    assert u == oracle.philox([43, 14, 2, 4], 99, 0)[2]


def test_splitmix64_weyl_structure():
    # splitmix64 output k of state s equals output 0 of state s + k*gamma
    gamma = 0x9E3779B97F4A7C15
    s0 = 0x1234
    seq = oracle.sm64_stream(s0, 5)
    for k in range(5):
        assert oracle.sm64_stream((s0 + k * gamma) & (2 ** 64 - 1), 1)[0] == seq[k]
    assert len(set(seq)) == 5


def test_schedules_closed_forms():
    lin = oracle.schedule(0, 0.1, 3.0, 256)
    assert lin[0] == 0.1 and abs(lin[-1] - 3.0) < 1e-15
    np.testing.assert_allclose(np.diff(lin), (3.0 - 0.1) / 255, rtol=1e-12)
    geo = oracle.schedule(1, 0.2, 3.0, 32)
    assert geo[0] == 0.2 and abs(geo[-1] - 3.0) < 1e-14
    np.testing.assert_allclose(geo[1:] / geo[:-1], 15.0 ** (1 / 31), rtol=1e-12)
    assert list(oracle.schedule(0, 0.7, 9.0, 1)) == [0.7]


def _exact_threshold(x):
    """floor(exp(-x) 2^32) clamped to 2^32-1, in 60-digit decimal, plus the
    distance of exp(-x) 2^32 from the nearest integer."""
    getcontext().prec = 60
    v = (-Decimal(x)).exp() * Decimal(2 ** 32)
    f = int(v)
    return min(f, 2 ** 32 - 1), float(min(v - f, f + 1 - v))


@pytest.mark.parametrize("beta", [0.0, 0.1, 0.37, 1.0, 2.5, 3.0, 11.0, 40.0])
def test_metropolis_thresholds_match_exact_quantisation(beta):
    K = 24
    thr = oracle.thresholds(np.array([beta]), K)[0]
    for k in range(1, K + 1):
        exact, dist = _exact_threshold(Decimal(2 * k) * Decimal(beta))
        if dist > 1e-4:
            assert int(thr[k - 1]) == exact, (beta, k)
    assert np.all(np.diff(thr.astype(np.int64)) <= 0)
    if beta == 0.0:
        assert np.all(thr == 0xFFFFFFFF)


def test_exchange_thresholds_match_exact_quantisation():
    beta = oracle.schedule(1, 0.2, 3.0, 32)
    M = 640
    thrx = oracle.exchange_thresholds(beta, M)
    for k in (0, 7, 30):
        db = Decimal(float(beta[k + 1] - beta[k]))
        for m in (1, 2, 5, 44, 45, 100, 606, 607, 608, 640):
            exact, dist = _exact_threshold(Decimal(2 * m) * db)
            if dist > 1e-4:
                assert int(thrx[k, m - 1]) == exact, (k, m)
    # the last nonzero entry of the lowest and highest pair (the table
    # lengths for this ladder)
    assert np.nonzero(thrx[0])[0].max() + 1 == 607
    assert np.nonzero(thrx[30])[0].max() + 1 == 44
