"""Pins of the oracle's instance generator and energy (Sec. II tile planting,
Eq. 1).  Each check compares the oracle with something other than itself:
exhaustive enumeration by an independent helper, the planting argument,
gauge invariance, or the lattice bookkeeping of this file."""
import numpy as np
import pytest

import oracle
from conftest import bonds_from_J, neighbours


@pytest.mark.parametrize("L,cls,seed", [(4, 6, 1), (4, 2, 7), (6, 6, 3), (8, 6, 11), (8, 4, 5),
                                        (10, 6, 99), (12, 0, 2), (16, -1, 42)])
def test_planted_energy_equals_sum_of_tile_minima(L, cls, seed):
    # planting argument: H = sum_t H_t and the planted state minimises every
    # H_t, so E(planted) is exactly the sum of the tile minima the generator
    # reports as E_gs.
    J, g, egs = oracle.make_instance(L, cls, seed)
    assert egs < 0
    assert oracle.energy(J, g, (L, L, L)) == egs
    assert oracle.epsilon(egs, egs) == 0.0


@pytest.mark.parametrize("L,seed", [(4, 5), (6, 8), (12, 13)])
def test_coupling_layout_consistent_and_in_range(L, seed):
    J, g, egs = oracle.make_instance(L, 6, seed)
    nbr = neighbours((L, L, L))
    assert J.min() >= -4 and J.max() <= 4
    # J[-d][i] == J[+d][nbr(i, -d)] for every direction pair
    for d in (0, 2, 4):
        np.testing.assert_array_equal(J[d + 1], J[d][nbr[d + 1]])


@pytest.mark.parametrize("dims,seed,cls", [((3, 3, 2), 1, 6), ((3, 3, 2), 2, 2),
                                           ((3, 3, 3), 3, 6), ((3, 3, 3), 4, 4),
                                           ((2, 2, 2), 5, 6), ((4, 3, 2), 6, -1)])
def test_bruteforce_ground_state_open_boxes(dims, seed, cls, bruteforce):
    # exhaustive enumeration of all 2^N states of a tiny open box built from
    # whole tiles: the minimum equals the generator's E_gs and the planted
    # configuration attains it
    J, g, egs = oracle.make_instance(0, cls, seed, dims=dims, periodic=False)
    N = dims[0] * dims[1] * dims[2]
    emin, dos = bruteforce(N, bonds_from_J(J, dims))
    assert emin == egs
    assert oracle.energy(J, g, dims) == egs
    assert sum(dos.values()) == 2 ** N


def test_energy_matches_enumeration_on_every_state(bruteforce):
    # the oracle's Eq. (1) energy over all 4096 states of a 3x2x2 box equals
    # the independent helper's density of states, state by state in count
    dims = (3, 2, 2)
    rng = np.random.default_rng(0)
    N = 12
    J = np.zeros((6, N), np.int8)
    nbr = neighbours(dims)
    for i in range(N):
        x, y, z = i % 3, (i // 3) % 2, i // 6
        if x < 2:
            J[0, i] = rng.integers(-4, 5)
        if y < 1:
            J[2, i] = rng.integers(-4, 5)
        if z < 1:
            J[4, i] = rng.integers(-4, 5)
    for d in (0, 2, 4):
        J[d + 1] = J[d][nbr[d + 1]]
    counts = {}
    for n in range(2 ** N):
        s = np.array([-1 if (n >> b) & 1 else 1 for b in range(N)], np.int8)
        E = oracle.energy(J, s, dims)
        counts[E] = counts.get(E, 0) + 1
    _, dos = bruteforce(N, bonds_from_J(J, dims))
    assert counts == dos


@pytest.mark.parametrize("L,seed", [(4, 21), (8, 22)])
def test_gauge_invariance(L, seed):
    # undoing the generator's gauge gamma (= planted state) must give a
    # coupling set whose all-(+1) state has energy E_gs, and E_J(gamma*s) ==
    # E_{J0}(s) for random s
    J, g, egs = oracle.make_instance(L, 6, seed)
    nbr = neighbours((L, L, L))
    J0 = (J.astype(np.int32) * g[None, :] * g[nbr]).astype(np.int8)
    ones = np.ones(L ** 3, np.int8)
    assert oracle.energy(J0, ones, (L, L, L)) == egs
    rng = np.random.default_rng(seed)
    for _ in range(5):
        s = rng.choice(np.array([-1, 1], np.int8), L ** 3)
        assert oracle.energy(J, (g * s).astype(np.int8), (L, L, L)) == oracle.energy(J0, s, (L, L, L))


def test_generator_is_deterministic_and_seed_sensitive():
    a = oracle.make_instance(8, 6, 123)
    b = oracle.make_instance(8, 6, 123)
    c = oracle.make_instance(8, 6, 124)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[2] == b[2]
    assert not np.array_equal(a[0], c[0])


def test_planted_state_is_gauge_scrambled():
    # the planted configuration is a random gauge, not all-(+1)
    J, g, egs = oracle.make_instance(8, 6, 77)
    frac = float(np.mean(g == 1))
    assert 0.4 < frac < 0.6


def test_random_configurations_average_epsilon_one():
    # the random-configuration baseline of Sec. I.A (about 100 % off): a
    # uniformly random configuration has E[E] = 0, so E[eps] = 1; check the
    # sample mean against a CLT bound
    L = 8
    J, g, egs = oracle.make_instance(L, 6, 31)
    n = 2000
    Es = np.array([oracle.energy(J, oracle.init_spins(L, 0xABC, 3, r), (L, L, L))
                   for r in range(n)], np.float64)
    var_E = float(np.sum(J[[0, 2, 4]].astype(np.float64) ** 2))  # Var E = sum_bonds J^2
    assert abs(Es.mean()) < 5.0 * np.sqrt(var_E / n)
    eps = np.array([oracle.epsilon(int(e), egs) for e in Es])
    assert abs(eps.mean() - 1.0) < 5.0 * np.sqrt(var_E / n) / abs(egs)
    assert abs(Es.var() / var_E - 1.0) < 0.15


def _single_tile_faces(J):
    """Frustrated faces of the one tile of an open 2x2x2 box, from J alone.

    Site i = x + 2 (y + 2 z).  Each face of the cube is a plaquette of four
    bonds; it is frustrated when the product of their couplings is negative.
    The product is invariant under any gauge s_i -> g_i s_i, so the count
    read from the scrambled J equals the count of the tile as drawn."""
    def site(x, y, z):
        return x + 2 * (y + 2 * z)

    def bx(y, z):
        return int(J[0, site(0, y, z)])

    def by(x, z):
        return int(J[2, site(x, 0, z)])

    def bz(x, y):
        return int(J[4, site(x, y, 0)])

    plaquettes = []
    for x in (0, 1):   # faces normal to x: y- and z-bonds at that x
        plaquettes.append((by(x, 0), bz(x, 1), by(x, 1), bz(x, 0)))
    for y in (0, 1):   # normal to y: x- and z-bonds at that y
        plaquettes.append((bx(y, 0), bz(1, y), bx(y, 1), bz(0, y)))
    for z in (0, 1):   # normal to z: x- and y-bonds at that z
        plaquettes.append((bx(0, z), by(1, z), bx(1, z), by(0, z)))
    return sum(1 for p in plaquettes if np.prod(np.sign(p)) < 0)


@pytest.mark.parametrize("cls", [0, 2, 4, 6])
@pytest.mark.parametrize("seed", [1, 2, 3, 17, 2025])
def test_tile_class_filter_counts_frustrated_faces(cls, seed):
    # A 2x2x2 open box holds exactly one tile, so every bond carries one tile
    # coupling: its twelve couplings are nonzero and in [-2, 2], and the
    # number of frustrated faces, counted here from J by plaquette products,
    # is the class the generator was asked for (Sec. II: classes differ by
    # the frustration of their tiles).
    J, g, egs = oracle.make_instance(0, cls, seed, dims=(2, 2, 2), periodic=False)
    bonds = [int(J[0, x + 2 * (y + 2 * z)]) for y in (0, 1) for z in (0, 1) for x in (0,)]
    bonds += [int(J[2, x + 2 * (0 + 2 * z)]) for x in (0, 1) for z in (0, 1)]
    bonds += [int(J[4, x + 2 * (y + 0)]) for x in (0, 1) for y in (0, 1)]
    assert len(bonds) == 12
    assert all(b != 0 for b in bonds)
    assert all(abs(b) <= 2 for b in bonds)
    # no coupling outside the twelve cube edges
    assert int(np.count_nonzero(J)) == 24
    assert _single_tile_faces(J) == cls


def test_unfiltered_tiles_reach_every_even_face_count():
    # with no class filter (-1) the draws cover all four possible counts and
    # never an odd one (every cube has an even number of frustrated faces)
    seen = set()
    for seed in range(200):
        J, g, egs = oracle.make_instance(0, -1, seed, dims=(2, 2, 2), periodic=False)
        seen.add(_single_tile_faces(J))
    assert seen == {0, 2, 4, 6}
