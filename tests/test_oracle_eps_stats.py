"""Pins of the oracle's optimality-gap statistics (Eq. 2 and the TT-eps
criterion of App. D: the mean gap over the trials of an instance, how many
trials reach a target, and a histogram of the gap).

The energies are constructed so that every answer is known by construction:
with E_gs = -1024 the gap of E_gs + k is k / 1024, exactly representable, so
targets m / 1024 split the trials at known places and a histogram of 1024
bins over [0, 1) puts trial k in bin k.  A wrong comparison (< for <=), an
off-by-one bin, a wrong group offset or a dropped term fails one of these.
"""
import numpy as np
import pytest

import oracle


def test_ground_state_trials():
    # every trial at E_gs: sum n E_gs, eps 0 everywhere, all in bin 0
    n, egs = 37, -5000
    e = np.full((1, n), egs, np.int32)
    st = oracle.eps_stats(e, egs, targets=(0.0, 0.01), eps_max=0.1, n_bins=10)
    assert st["sum"][0] == n * egs
    assert st["emin"][0] == egs and st["emax"][0] == egs
    assert st["n_le"][0].tolist() == [n, n]
    assert st["hist"][0].tolist() == [n] + [0] * 9


def test_counts_and_bins_by_construction():
    egs = -1024
    rng = np.random.default_rng(5)
    ks = rng.integers(0, 1024, size=500)
    e = (egs + ks).astype(np.int32)[None, :]
    targets = [m / 1024 for m in (0, 1, 30, 31, 512, 1023)]
    st = oracle.eps_stats(e, egs, targets=targets, eps_max=1.0, n_bins=1024)
    for t, m in zip(targets, (0, 1, 30, 31, 512, 1023)):
        assert st["n_le"][0][targets.index(t)] == int(np.sum(ks <= m))
    assert st["hist"][0].tolist() == np.bincount(ks, minlength=1024).tolist()
    assert st["sum"][0] == int(np.sum(egs + ks.astype(np.int64)))
    assert st["emin"][0] == egs + ks.min() and st["emax"][0] == egs + ks.max()


def test_clamping_below_and_above_the_range():
    # E below E_gs (a negative gap) lands in bin 0 and counts for every
    # target >= 0; gaps at or above eps_max land in the last bin
    egs = -1024
    ks = np.array([-3, -1, 0, 255, 256, 1024, 5000], np.int64)
    e = (egs + ks).astype(np.int32)[None, :]
    st = oracle.eps_stats(e, egs, targets=(0.0,), eps_max=0.25, n_bins=4)
    # eps = k/1024; bin = floor(eps / 0.25 * 4) = floor(k / 64), clamped to [0, 3]
    assert st["hist"][0].tolist() == [3, 0, 0, 4]
    assert st["n_le"][0].tolist() == [3]


def test_groups_are_independent_and_use_their_own_ground_state():
    rng = np.random.default_rng(9)
    G, n = 6, 50
    egs = np.array([-1024, -2048, -512, -1024, -4096, -1024], np.int64)
    ks = rng.integers(0, 200, size=(G, n))
    e = (egs[:, None] + ks).astype(np.int32)
    st = oracle.eps_stats(e, egs, targets=(0.05,), eps_max=0.5, n_bins=8)
    for g in range(G):
        one = oracle.eps_stats(e[g:g + 1], egs[g], targets=(0.05,), eps_max=0.5, n_bins=8)
        assert st["sum"][g] == one["sum"][0]
        assert st["n_le"][g].tolist() == one["n_le"][0].tolist()
        assert st["hist"][g].tolist() == one["hist"][0].tolist()
        # the target 0.05 is 0.05 |E_gs| energy units above E_gs
        assert st["n_le"][g][0] == int(np.sum(ks[g] <= 0.05 * abs(egs[g])))


def test_invariants_on_annealed_energies():
    # on real anneal output: the histogram holds every trial, counts grow
    # with the target, the statistics do not depend on trial order
    L = 6
    J, g, egs = oracle.make_instance(L, 6, 404)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 20), 24)
    _, E, _ = oracle.sa_run(L, J, 77, 0, thr, n_rep=40)
    e = E.astype(np.int32)[None, :]
    tg = (0.0, 0.02, 0.05, 0.1, 1.0)
    st = oracle.eps_stats(e, egs, targets=tg, eps_max=0.2, n_bins=16)
    assert int(st["hist"].sum()) == 40
    assert list(st["n_le"][0]) == sorted(st["n_le"][0])
    perm = np.random.default_rng(1).permutation(40)
    st2 = oracle.eps_stats(e[:, perm], egs, targets=tg, eps_max=0.2, n_bins=16)
    for k in ("sum", "emin", "emax", "n_le", "hist"):
        np.testing.assert_array_equal(st[k], st2[k])


def test_bad_input_is_rejected():
    with pytest.raises(RuntimeError):
        oracle.eps_stats(np.zeros((1, 3), np.int32), 0, targets=(0.1,))
    with pytest.raises(RuntimeError):
        oracle.eps_stats(np.zeros((1, 3), np.int32), -5, targets=(0.1,), eps_max=0.0, n_bins=4)
