"""Pins of the oracle's Metropolis sweep (App. D simulated annealing) and
replica exchange (App. D parallel tempering).

The strongest pins are statistical: at fixed beta the sweep must sample the
Boltzmann law p(s) ~ exp(-beta H(s)) of App. A, and two exchanging walkers
must sample the product of their two Boltzmann laws; the exact laws come
from exhaustive enumeration by an independent helper.  The rest are
invariants and closed-form special cases."""
import numpy as np
import pytest
from scipy import stats

import oracle
from conftest import bonds_from_J, neighbours

K = 24


def _embedded_block(seed, block=(2, 2, 2), L=4):
    """Random J in [-4, 4] on the bonds of a small open block inside an L^3
    periodic lattice; every other coupling is zero.  Returns J and the list
    of block sites."""
    rng = np.random.default_rng(seed)
    N = L ** 3
    J = np.zeros((6, N), np.int8)
    nbr = neighbours((L, L, L))
    bx, by, bz = block
    sites = []
    for z in range(bz):
        for y in range(by):
            for x in range(bx):
                i = x + L * (y + L * z)
                sites.append(i)
                if x + 1 < bx:
                    J[0, i] = rng.integers(-4, 5)
                if y + 1 < by:
                    J[2, i] = rng.integers(-4, 5)
                if z + 1 < bz:
                    J[4, i] = rng.integers(-4, 5)
    for d in (0, 2, 4):
        J[d + 1] = J[d][nbr[d + 1]]
    return J, sites


def _boltzmann(dos, beta):
    Es = np.array(sorted(dos))
    w = np.array([dos[e] for e in Es], np.float64) * np.exp(-beta * (Es - Es.min()))
    return Es, w / w.sum()


def _chi2_pvalue(samples, Es, p, n):
    counts = np.array([np.sum(samples == e) for e in Es], np.float64)
    assert counts.sum() == n, "sample outside the enumerated spectrum"
    exp = p * n
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] < 5:
        obs[-2] += obs[-1]
        ex[-2] += ex[-1]
        obs, ex = obs[:-1], ex[:-1]
    return stats.chisquare(obs, ex).pvalue


def _exact_samples(J, L, sites, beta, n, rng):
    """n configurations of the L^3 lattice whose coupled block is an exact
    Boltzmann sample at beta (by enumeration of its 2^8 states); the free
    spins are uniform."""
    idx = {s: k for k, s in enumerate(sites)}
    bonds = [(idx[i], idx[j], v) for (i, j, v) in bonds_from_J(J, (L, L, L))]
    nb = len(sites)
    states = np.array([[-1 if (m >> b) & 1 else 1 for b in range(nb)] for m in range(2 ** nb)])
    E = np.zeros(2 ** nb)
    for (i, j, v) in bonds:
        E += v * states[:, i] * states[:, j]
    w = np.exp(-beta * (E - E.min()))
    pick = rng.choice(2 ** nb, size=n, p=w / w.sum())
    out = rng.choice(np.array([-1, 1], np.int8), size=(n, L ** 3))
    out[:, sites] = states[pick]
    return np.ascontiguousarray(out.astype(np.int8))


def _stationarity_pvalue(J, L, sites, beta_law, thr, n, seed, bruteforce):
    _, dos = _enumerate_block(J, L, sites, bruteforce)
    Es, p = _boltzmann(dos, beta_law)
    rng = np.random.default_rng(seed)
    s0 = _exact_samples(J, L, sites, beta_law, n, rng)
    _, en, _ = oracle.sa_run(L, J, 0xC0FFEE + seed, 9, thr, n_rep=n, spins=s0)
    return _chi2_pvalue(en, Es, p, n)


@pytest.mark.parametrize("beta,seed", [(0.3, 1), (0.8, 2)])
def test_fixed_beta_sweeps_keep_boltzmann_law(beta, seed, bruteforce):
    # stationarity: started from exact Boltzmann samples at beta, eight
    # sweeps at the same beta must leave the energy law unchanged
    L = 4
    J, sites = _embedded_block(seed)
    thr = oracle.thresholds(np.full(8, beta), K)
    pval = _stationarity_pvalue(J, L, sites, beta, thr, 12000, seed, bruteforce)
    assert pval > 1e-3, pval


def test_boltzmann_check_detects_a_wrong_acceptance(bruteforce):
    # negative control: the same check applied to sweeps whose acceptance
    # table was built for beta/2 (the classic dE-vs-dE/2 slip) must fail
    L = 4
    beta = 0.8
    J, sites = _embedded_block(2)
    thr = oracle.thresholds(np.full(8, beta / 2), K)
    pval = _stationarity_pvalue(J, L, sites, beta, thr, 12000, 2, bruteforce)
    assert pval < 1e-6, pval


def _enumerate_block(J, L, sites, bruteforce):
    """Exhaustive density of states of the coupled block (sites relabelled)."""
    idx = {s: k for k, s in enumerate(sites)}
    bonds = [(idx[i], idx[j], v) for (i, j, v) in bonds_from_J(J, (L, L, L))]
    return bruteforce(len(sites), bonds)


def test_two_temperature_exchange_samples_product_law(bruteforce):
    L = 4
    J, sites = _embedded_block(5)
    _, dos = _enumerate_block(J, L, sites, bruteforce)
    betas = np.array([0.3, 0.9])
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 64)
    n_runs = 4000
    rng = np.random.default_rng(6)
    s_hot = _exact_samples(J, L, sites, betas[0], n_runs, rng)
    s_cold = _exact_samples(J, L, sites, betas[1], n_runs, rng)
    e_slot = np.zeros((2, n_runs), np.int64)
    for r in range(n_runs):
        start = np.stack([s_hot[r], s_cold[r]])
        out = oracle.pt_run(L, J, 0xBEEF, r, thr, thrx, n_steps=9, spins=start,
                            pos=np.array([0, 1], np.int32))
        for w in range(2):
            e_slot[out["pos"][w], r] = out["energy"][w]
    for k in range(2):
        Es, p = _boltzmann(dos, betas[k])
        assert _chi2_pvalue(e_slot[k], Es, p, n_runs) > 1e-3, k
    # the exchange must matter: the colder slot holds the lower energies
    assert e_slot[1].mean() < e_slot[0].mean()


@pytest.mark.parametrize("L,seed", [(4, 3), (6, 4), (8, 5)])
def test_tracked_energy_equals_recomputed_after_every_sweep(L, seed):
    J, g, egs = oracle.make_instance(L, 6, seed)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 40), K)
    sp, en, em = oracle.sa_run(L, J, 17, 2, thr, n_rep=3, want_emin=True, check=True)
    for r in range(3):
        assert en[r] == oracle.energy(J, sp[r], (L, L, L))
        assert em[r] <= en[r]
        assert em[r] >= egs


def test_pt_tracked_energy_and_permutation():
    L = 6
    J, g, egs = oracle.make_instance(L, 6, 8)
    betas = oracle.schedule(1, 0.2, 3.0, 8)
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 400)
    out = oracle.pt_run(L, J, 3, 1, thr, thrx, n_steps=30, want_trace=True, want_swaps=True,
                        check=True)
    assert sorted(out["pos"]) == list(range(8))
    for w in range(8):
        assert out["energy"][w] == oracle.energy(J, out["spins"][w], (L, L, L))
    assert out["emin_trace"][-1] == out["energy"].min()
    assert np.all(out["emin_trace"] >= egs)
    assert out["swap_acc"].sum() > 0


def test_local_field_gives_flip_energy_change():
    # dE(flip i) = -2 s_i h_i: the oracle's local field against its energy
    rng = np.random.default_rng(4)
    L = 4
    nbr = neighbours((L, L, L))
    for _ in range(20):
        J = np.zeros((6, L ** 3), np.int8)
        for d in (0, 2, 4):
            J[d] = rng.integers(-4, 5, L ** 3)
            J[d + 1] = J[d][nbr[d + 1]]
        s = rng.choice(np.array([-1, 1], np.int8), L ** 3)
        i = int(rng.integers(L ** 3))
        h = oracle.local_field(J, s, (L, L, L), i)
        s2 = s.copy()
        s2[i] = -s2[i]
        assert oracle.energy(J, s2, (L, L, L)) - oracle.energy(J, s, (L, L, L)) == -2 * s[i] * h


def test_zero_temperature_is_greedy_descent():
    # beta = infinity (all thresholds zero): only dE <= 0 moves, so the
    # energy never rises and the best-seen energy is the final one
    L = 8
    J, g, egs = oracle.make_instance(L, 6, 12)
    thr = np.zeros((1, K), np.uint32)
    sp = None
    E_prev = None
    for s in range(6):
        sp, en, _ = oracle.sa_run(L, J, 5, 0, thr, n_rep=1, sweep0=s, spins=sp)
        if E_prev is not None:
            assert en[0] <= E_prev
        E_prev = en[0]


def test_ferromagnet_zero_temperature_heals_one_defect():
    # closed form: J = -1 on every bond, all spins +1 except one; at
    # beta = infinity one sweep restores all +1 (E = -3N) whichever colour
    # the defect has
    L = 4
    N = L ** 3
    J = -np.ones((6, N), np.int8)
    thr = np.zeros((1, K), np.uint32)
    for site in (0, 1, 21, 42):
        s = np.ones((1, N), np.int8)
        s[0, site] = -1
        sp, en, _ = oracle.sa_run(L, J, 1, 0, thr, n_rep=1, spins=s)
        assert en[0] == -3 * N
        assert np.all(sp == 1)


def test_infinite_temperature_flips_every_spin():
    # closed form: at beta = 0 the threshold is 2^32-1, so every proposal
    # is accepted (unless its word is exactly 2^32-1); one sweep maps s to -s
    L = 6
    J, g, egs = oracle.make_instance(L, 6, 13)
    thr = np.full((3, K), 0xFFFFFFFF, np.uint32)
    s0 = oracle.init_spins(L, 7, 1, 0)
    sp, en, _ = oracle.sa_run(L, J, 7, 1, thr, n_rep=1, spins=s0[None, :])
    np.testing.assert_array_equal(sp[0], -s0)
    assert en[0] == oracle.energy(J, s0, (L, L, L))


def test_order_inside_a_colour_does_not_matter():
    # same-colour sites share no bond, so visiting them in reverse order
    # yields the same chain bit for bit
    for L in (4, 6, 10):
        J, g, egs = oracle.make_instance(L, 6, L)
        thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 20), K)
        a = oracle.sa_run(L, J, 21, 3, thr, n_rep=2)
        b = oracle.sa_run(L, J, 21, 3, thr, n_rep=2, reversed_order=True)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_resume_equals_uninterrupted_run():
    L = 8
    J, g, egs = oracle.make_instance(L, 6, 14)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 30), K)
    full = oracle.sa_run(L, J, 33, 5, thr, n_rep=2)
    part = oracle.sa_run(L, J, 33, 5, thr[:11], n_rep=2)
    rest = oracle.sa_run(L, J, 33, 5, thr[11:], n_rep=2, sweep0=11, spins=part[0])
    np.testing.assert_array_equal(full[0], rest[0])
    np.testing.assert_array_equal(full[1], rest[1])
    # PT: 17 steps == 10 + 7
    betas = oracle.schedule(1, 0.2, 3.0, 4)
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 300)
    a = oracle.pt_run(6, oracle.make_instance(6, 6, 2)[0], 4, 2, thr, thrx, 17)
    J6 = oracle.make_instance(6, 6, 2)[0]
    b1 = oracle.pt_run(6, J6, 4, 2, thr, thrx, 10)
    b2 = oracle.pt_run(6, J6, 4, 2, thr, thrx, 7, step0=10, spins=b1["spins"], pos=b1["pos"])
    np.testing.assert_array_equal(a["spins"], b2["spins"])
    np.testing.assert_array_equal(a["pos"], b2["pos"])


def test_equal_temperatures_always_exchange():
    # closed form: beta_0 == beta_1 gives exchange threshold 2^32-1, so the
    # pair (0, 1), active on even steps, swaps on every even step (the table
    # spans every energy difference an L=4 instance can show)
    L = 4
    J, g, egs = oracle.make_instance(L, 6, 15)
    betas = np.array([0.7, 0.7])
    out = oracle.pt_run(L, J, 9, 0, oracle.thresholds(betas, K),
                        oracle.exchange_thresholds(betas, 800), n_steps=11, want_swaps=True)
    assert out["swap_acc"][0] == 6


def test_init_stream_is_balanced_and_replica_dependent():
    L = 8
    a = oracle.init_spins(L, 1, 0, 0)
    b = oracle.init_spins(L, 1, 0, 1)
    assert set(np.unique(a)) == {-1, 1}
    assert not np.array_equal(a, b)
    ups = sum(int(np.sum(oracle.init_spins(L, 1, 0, r) == 1)) for r in range(20))
    n = 20 * L ** 3
    assert abs(ups - n / 2) < 5 * np.sqrt(n / 4)
