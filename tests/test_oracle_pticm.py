"""Pins of the oracle's parallel tempering with isoenergetic cluster moves
(App. D: PT+ICM; the move is Houdayer's two-replica cluster move).

  * the cluster move equals an independent construction: seed chosen by the
    stated rule, cluster = connected component of the disagreeing sites in
    the graph of nonzero couplings (scipy), both walkers flipped on it; the
    summed energy of the two walkers is unchanged;
  * without cluster moves, copy 0 is exactly the PT chain;
  * stationarity: started from exact Boltzmann samples at each slot's beta,
    PT+ICM steps keep every walker's energy law and the joint law of the two
    copies at one slot equal to the (product of) Boltzmann laws, from
    enumeration by the independent helper (chi-square);
  * tracked energies equal recomputed ones.
"""
import numpy as np
import pytest
from scipy import sparse, stats
from scipy.sparse import csgraph

import oracle
from conftest import neighbours
from test_oracle_metropolis import _boltzmann, _chi2_pvalue, _embedded_block, _enumerate_block, _exact_samples

K = 24


def _column_order(L):
    """Sites in the order (colour, column, height) of the colour-split
    column layout, from this file's own arithmetic."""
    H = L // 2
    out = []
    for c in range(2):
        for col in range(H * L):
            y, k = col // H, col % H
            for z in range(L):
                x = 2 * k + ((y + z + c) & 1)
                out.append(x + L * (y + L * z))
    return out


def _expected_move(L, J, sa, sb, u):
    N = L ** 3
    neg = sa != sb
    order = [i for i in _column_order(L) if neg[i]]
    if not order:
        return sa.copy(), sb.copy(), 0
    seed = order[(u * len(order)) >> 32]
    nbr = neighbours((L, L, L))
    rows, cols = [], []
    for d in range(6):
        for i in range(N):
            j = nbr[d][i]
            if J[d, i] != 0 and neg[i] and neg[j]:
                rows.append(i)
                cols.append(j)
    g = sparse.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    _, lab = csgraph.connected_components(g, directed=False)
    cl = (lab == lab[seed]) & neg
    a, b = sa.copy(), sb.copy()
    a[cl] = -a[cl]
    b[cl] = -b[cl]
    return a, b, int(cl.sum())


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_cluster_move_is_the_connected_component_and_isoenergetic(seed):
    rng = np.random.default_rng(seed)
    L = 6
    J, _, _ = oracle.make_instance(L, 6, 50 + seed)
    J = J.reshape(6, -1).copy()
    # knock out some bonds (both directions) so that zero couplings matter
    nbr = neighbours((L, L, L))
    for i in rng.choice(L ** 3, 40, replace=False):
        d = int(rng.integers(0, 3)) * 2
        J[d, i] = 0
        J[d + 1, nbr[d][i]] = 0
    for trial in range(10):
        sa = rng.choice(np.array([-1, 1], np.int8), L ** 3)
        sb = sa.copy()
        flip = rng.random(L ** 3) < rng.uniform(0.05, 0.6)
        sb[flip] = -sb[flip]
        u = int(rng.integers(0, 2 ** 32))
        a, b, n = oracle.icm_move(L, J, sa, sb, u)
        ea, eb, ne = _expected_move(L, J, sa, sb, u)
        np.testing.assert_array_equal(a, ea)
        np.testing.assert_array_equal(b, eb)
        assert n == ne
        dims = (L, L, L)
        assert oracle.energy(J, a, dims) + oracle.energy(J, b, dims) == \
            oracle.energy(J, sa, dims) + oracle.energy(J, sb, dims)
    # identical walkers: no move
    a, b, n = oracle.icm_move(L, J, sa, sa, 123)
    assert n == 0 and np.array_equal(a, sa)


def test_without_cluster_moves_copy_zero_is_parallel_tempering():
    L, T = 6, 6
    J, _, _ = oracle.make_instance(L, 6, 9)
    betas = oracle.schedule(1, 0.2, 3.0, T)
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 300)
    a = oracle.pticm_run(L, J, 7, 3, thr, thrx, n_steps=25, icm_from=T, want_swaps=True)
    p = oracle.pt_run(L, J, 7, 3, thr, thrx, n_steps=25, want_swaps=True)
    np.testing.assert_array_equal(a["spins"][:T], p["spins"])
    np.testing.assert_array_equal(a["energy"][:T], p["energy"])
    np.testing.assert_array_equal(a["pos"][:T], p["pos"])
    np.testing.assert_array_equal(a["swap_acc"][:T - 1], p["swap_acc"])


def test_tracked_energies_and_cluster_moves_happen():
    L, T = 6, 8
    J, _, egs = oracle.make_instance(L, 6, 10)
    betas = oracle.schedule(1, 0.2, 3.0, T)
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 400)
    out = oracle.pticm_run(L, J, 11, 0, thr, thrx, n_steps=40, icm_from=2, want_trace=True,
                           want_swaps=True, want_icm=True, check=True)
    for w in range(2 * T):
        assert out["energy"][w] == oracle.energy(J, out["spins"][w], (L, L, L))
    for cp in range(2):
        assert sorted(out["pos"][cp * T:(cp + 1) * T]) == list(range(T))
    assert out["icm_flipped"].sum() > 0
    assert np.all(out["emin_trace"] >= egs)


def test_pticm_keeps_boltzmann_laws(bruteforce):
    # two slots (beta 0.3 and 0.9), two copies, cluster moves at both slots;
    # every walker starts from an exact Boltzmann sample at its slot
    L = 4
    J, sites = _embedded_block(5)
    _, dos = _enumerate_block(J, L, sites, bruteforce)
    betas = np.array([0.3, 0.9])
    thr = oracle.thresholds(betas, K)
    thrx = oracle.exchange_thresholds(betas, 64)
    n_runs = 4000
    rng = np.random.default_rng(16)
    starts = [_exact_samples(J, L, sites, betas[k], n_runs, rng) for k in (0, 1, 0, 1)]
    e = np.zeros((2, 2, n_runs), np.int64)   # copy, slot, run
    for r in range(n_runs):
        out = oracle.pticm_run(L, J, 0xFACE, r, thr, thrx, n_steps=7, icm_from=0,
                               spins=np.stack([s[r] for s in starts]),
                               pos=np.array([0, 1, 0, 1], np.int32))
        for w in range(4):
            e[w // 2, out["pos"][w], r] = out["energy"][w]
    for cp in range(2):
        for k in range(2):
            Es, p = _boltzmann(dos, betas[k])
            assert _chi2_pvalue(e[cp, k], Es, p, n_runs) > 1e-3, (cp, k)
    # joint law of the two copies at the cold slot: the product law
    Es, p = _boltzmann(dos, betas[1])
    idx = {E: i for i, E in enumerate(Es)}
    obs = np.zeros((len(Es), len(Es)))
    for a, b in zip(e[0, 1], e[1, 1]):
        obs[idx[a], idx[b]] += 1
    exp = np.outer(p, p) * n_runs
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    x = np.append(exp[keep], exp[~keep].sum())
    assert stats.chisquare(o, x).pvalue > 1e-3
