"""Pins of the oracle's fragment decimation: the bootstrapped subsystem
optimisation of Sec. I with fixed-sweep simulated annealing as the subsystem
optimiser, on cubic fragments that overlap earlier decimations (App. C).

The method is a heuristic, so the oracle is its steps written out; what pins
those steps here:
  * one fragment anneal reaches the exact minimum of the fragment's energy
    (in-fragment bonds, decimated sites as fixed boundary spins), found by
    exhaustive enumeration in an independent helper;
  * single-site fragments carry no bond: every proposal flips, so the
    decimated spin is the init-stream spin times (-1)^S (closed form over
    the Philox words, which are themselves pinned to rocRAND);
  * at beta = infinity a spin whose whole fragment was decimated before it
    ends anti-aligned with its local field (closed form of greedy descent);
  * the order of the cores inside a phase does not change the result;
  * every output spin is +-1 and the energy is that of Eq. 1.
"""
import numpy as np
import pytest

import oracle

K = 24


def _geometry(L, core, halo, k):
    """The test's own fragment geometry: global site of every local site
    j = lx + l (ly + l lz) of core k's fragment."""
    l = core + 2 * halo
    nb = L // core
    bx, by, bz = k % nb, (k // nb) % nb, k // (nb * nb)
    g = []
    for lz in range(l):
        for ly in range(l):
            for lx in range(l):
                x = (bx * core - halo + lx) % L
                y = (by * core - halo + ly) % L
                z = (bz * core - halo + lz) % L
                g.append(x + L * (y + L * z))
    return l, g


def _fragment_problem(L, J, core, halo, k, dec):
    """Free spins of the fragment as a bond list over free spins plus one
    ghost spin (fixed boundary spins become bonds to the ghost, which the
    global flip symmetry lets us hold at +1), and the constant energy of
    bonds between two fixed spins."""
    N = L ** 3
    l, g = _geometry(L, core, halo, k)
    J = np.asarray(J).reshape(6, N)
    free = {j: n for n, j in enumerate(j for j in range(l ** 3) if dec[g[j]] == 0)}
    ghost = len(free)
    bonds, const = [], 0
    for j in range(l ** 3):
        lx, ly, lz = j % l, (j // l) % l, j // (l * l)
        for d, (dx, dy, dz) in ((0, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1))):
            mx, my, mz = lx + dx, ly + dy, lz + dz
            if mx >= l or my >= l or mz >= l:
                continue
            m = mx + l * (my + l * mz)
            Jb = int(J[d, g[j]])
            if Jb == 0:
                continue
            a_free, b_free = j in free, m in free
            if a_free and b_free:
                bonds.append((free[j], free[m], Jb))
            elif a_free:
                bonds.append((free[j], ghost, Jb * int(dec[g[m]])))
            elif b_free:
                bonds.append((free[m], ghost, Jb * int(dec[g[j]])))
            else:
                const += Jb * int(dec[g[j]]) * int(dec[g[m]])
    return ghost + 1, bonds, const, g


def _frag_energy(L, J, core, halo, k, frag):
    N = L ** 3
    l, g = _geometry(L, core, halo, k)
    J = np.asarray(J).reshape(6, N)
    E = 0
    for j in range(l ** 3):
        lx, ly, lz = j % l, (j // l) % l, j // (l * l)
        for d, step, ok in ((0, 1, lx + 1 < l), (2, l, ly + 1 < l), (4, l * l, lz + 1 < l)):
            if ok:
                E += int(J[d, g[j]]) * int(frag[j]) * int(frag[j + step])
    return E


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_fragment_anneal_reaches_the_enumerated_minimum(seed, bruteforce):
    # l = 3 fragments of an L = 8 instance with part of the fragment already
    # decimated (random fixed boundary spins).  No anneal may end below the
    # exact minimum of the fragment energy, and the best of 8 slow anneals
    # (what the decimation keeps) must reach it
    L, core, halo = 8, 1, 1
    J, _, _ = oracle.make_instance(L, 6, 1000 + seed)
    rng = np.random.default_rng(seed)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 6.0, 4000), K)
    for k in rng.choice(L ** 3, 3, replace=False):
        dec = np.zeros(L ** 3, np.int8)
        _, g = _geometry(L, core, halo, int(k))
        fixed = rng.choice(27, 9, replace=False)
        for j in fixed:
            dec[g[j]] = rng.choice([-1, 1])
        n, bonds, const, _ = _fragment_problem(L, J, core, halo, int(k), dec)
        emin, _ = bruteforce(n, bonds)
        energies = []
        for r in range(8):
            frag, E = oracle.frag_anneal(L, J, core, halo, int(k), r, seed, 3, thr, dec)
            assert E == _frag_energy(L, J, core, halo, int(k), frag)
            assert E >= emin + const
            # the fixed sites kept their values
            for j in fixed:
                assert frag[j] == dec[g[j]]
            energies.append(E)
        assert min(energies) == emin + const, (k, energies, emin + const)


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("S", [1, 2, 5])
def test_single_site_fragments_flip_every_sweep(order, S):
    # core 1, halo 0: a fragment is one spin with no bond; k_i = 0 always
    # flips, so the decimated spin is its init-stream value times (-1)^S
    L, seed, run = 6, 0x1234, 7
    J, _, _ = oracle.make_instance(L, 6, 5)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, S), K)
    dec = oracle.frag_decimate(L, J, 1, 0, 3, seed, run, thr, order=order)
    for i in range(L ** 3):
        w = oracle.philox([0, 0xFFFFFFFF, i, run], seed & 0xFFFFFFFF, seed >> 32)[0]
        s0 = -1 if (w >> 31) else 1
        assert dec[i] == s0 * (-1) ** S, i


def test_zero_temperature_last_phase_spins_oppose_their_field():
    # colour-class order with core 1, halo 1: the spins of the last class
    # (all coordinates odd) have every fragment neighbour decimated before
    # them; at beta = infinity they end anti-aligned with their local field
    # (or flipped S times from the init stream when the field is zero)
    L, S, seed, run = 8, 3, 99, 2
    J, _, _ = oracle.make_instance(L, 6, 321)
    thr = np.zeros((S, K), np.uint32)
    dec = oracle.frag_decimate(L, J, 1, 1, 2, seed, run, thr, order=0)
    Jr = J.reshape(6, -1)
    checked = 0
    for z in range(1, L, 2):
        for y in range(1, L, 2):
            for x in range(1, L, 2):
                i = x + L * (y + L * z)
                h = 0
                for d, (dx, dy, dz) in enumerate(((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                                  (0, 0, 1), (0, 0, -1))):
                    j = (x + dx) % L + L * (((y + dy) % L) + L * ((z + dz) % L))
                    h += int(Jr[d, i]) * int(dec[j])
                if h != 0:
                    assert dec[i] == -np.sign(h), i
                    checked += 1
                else:
                    # local index of the core in its 3^3 fragment is 13
                    w = oracle.philox([13, 0xFFFFFFFF, i, run], seed, 0)[0]
                    assert dec[i] == (-1 if (w >> 31) else 1) * (-1) ** S
    assert checked > 20


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("core,halo", [(1, 2), (3, 1), (2, 1), (2, 2)])
def test_order_inside_a_phase_does_not_matter(order, core, halo):
    L = 12
    J, _, _ = oracle.make_instance(L, 6, 77)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 6), K)
    a = oracle.frag_decimate(L, J, core, halo, 2, 5, 1, thr, order=order)
    b = oracle.frag_decimate(L, J, core, halo, 2, 5, 1, thr, order=order, reversed_order=True)
    np.testing.assert_array_equal(a, b)
    assert set(np.unique(a)) <= {-1, 1}


def test_outputs_and_argument_checks():
    L = 12
    J, _, egs = oracle.make_instance(L, 6, 8)
    thr = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, 20), K)
    dec = oracle.frag_decimate(L, J, 3, 1, 4, 9, 0, thr, order=1)
    assert set(np.unique(dec)) == {-1, 1}
    E = oracle.energy(J, dec, (L, L, L))
    assert E >= egs
    for core, halo, order in ((5, 1, 1), (1, 6, 1), (4, 1, 0)):   # L % c, l >= L, nb % P
        with pytest.raises(RuntimeError):
            oracle.frag_decimate(L, J, core, halo, 2, 9, 0, thr, order=order)
