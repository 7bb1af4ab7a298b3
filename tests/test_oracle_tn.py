"""Pins of the tensor-network fragment oracle (oracle/tn.py) against
things other than itself:

* exhaustive enumeration of the fragment's free spins (the definition of
  the conditional marginal, App. C) for small free sets, both variants;
* the closed form of a chain between a fixed spin and the centre
  (tanh of the effective coupling; its zero-temperature limit);
* symmetries: no fixed spin gives an exactly even marginal, gauge
  transformations leave it unchanged (or negate it at the centre), beta = 0
  gives zero, large beta approaches the tropical result;
* whole decimations of the uniform ferromagnet and antiferromagnet, whose
  ground states are known, and self-consistency of every decision.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import tn

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand_J(L, rng, jmax=4):
    """Consistent random couplings [6][N] (each bond stored twice)."""
    N = L ** 3
    J = np.zeros((6, N), np.int8)
    for i in range(N):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for d, (ex, ey, ez) in ((0, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1))):
            j = (x + ex) % L + L * (((y + ey) % L) + L * ((z + ez) % L))
            v = rng.integers(-jmax, jmax + 1)
            J[d, i] = v
            J[d + 1, j] = v
    return J


def _brute(L, J, dec, i, h, beta, tropical, s_centre):
    """Enumerate every assignment of the free sites (vectorised over the
    assignments), energy from the cube's bonds listed by coordinates."""
    x0, y0, z0 = i % L, (i // L) % L, i // (L * L)
    site = {}
    for dz in range(-h, h + 1):
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                site[(dx, dy, dz)] = (x0 + dx) % L + L * (((y0 + dy) % L) + L * ((z0 + dz) % L))
    free = [a for a in site.values() if a != i and dec[a] == 0]
    col = {a: k for k, a in enumerate(free)}
    n = len(free)
    cfg = 1 - 2 * ((np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1)   # [2^n, n] of +-1

    def spins(a):
        if a == i:
            return np.full(2 ** n, s_centre)
        return cfg[:, col[a]] if a in col else np.full(2 ** n, int(dec[a]))
    E = np.zeros(2 ** n, np.int64)
    for (dx, dy, dz), a in site.items():
        for d, (ex, ey, ez) in ((0, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1))):
            key = (dx + ex, dy + ey, dz + ez)
            if key in site:
                E += int(J[d, a]) * spins(a) * spins(site[key])
    if tropical:
        return int(E.min())
    w = -beta * E.astype(np.float64)
    top = w.max()
    return float(top + math.log(np.exp(w - top).sum()))


@pytest.mark.parametrize("h,n_free,seed", [(1, 6, 1), (1, 12, 2), (2, 10, 3), (2, 16, 4), (1, 18, 5)])
@pytest.mark.parametrize("tropical", [False, True])
def test_marginal_equals_enumeration(h, n_free, seed, tropical):
    L = 8
    rng = np.random.default_rng(seed)
    J = _rand_J(L, rng)
    i = int(rng.integers(L ** 3))
    l = 2 * h + 1
    x0, y0, z0 = i % L, (i // L) % L, i // (L * L)
    cube = [(x0 + dx) % L + L * (((y0 + dy) % L) + L * ((z0 + dz) % L))
            for dz in range(-h, h + 1) for dy in range(-h, h + 1) for dx in range(-h, h + 1)]
    others = [a for a in cube if a != i]
    dec = rng.choice(np.array([-1, 1], np.int8), L ** 3).astype(np.int8)
    free = rng.choice(len(others), size=min(n_free, len(others)), replace=False)
    for k in free:
        dec[others[k]] = 0
    for s in (1, -1):
        got = tn.site_value(L, J, dec, i, h, 2.0, tropical, s)
        ref = _brute(L, J, dec, i, h, 2.0, tropical, s)
        if tropical:
            assert got == ref
        else:
            assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref))
    assert l ** 3 == len(cube)


def test_chain_closed_form():
    # couplings only along the centre's x row; fixed spins at both row ends
    L, h, beta = 8, 2, 1.3
    rng = np.random.default_rng(7)
    N = L ** 3
    for trial in range(20):
        J = np.zeros((6, N), np.int8)
        i = int(rng.integers(N))
        x0, y0, z0 = i % L, (i // L) % L, i // (L * L)
        row = [(x0 + dx) % L + L * (y0 + L * z0) for dx in range(-h, h + 1)]
        js = rng.integers(-4, 5, size=2 * h)
        for k in range(2 * h):
            J[0, row[k]] = js[k]
            J[1, row[k + 1]] = js[k]
        # every other site fixed at random (their couplings are zero), the
        # row's inner sites and the centre's y and z neighbours free
        dec = rng.choice(np.array([-1, 1], np.int8), N).astype(np.int8)
        for k in range(1, 2 * h):
            dec[row[k]] = 0
        for ey, ez in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            dec[x0 + L * ((y0 + ey) % L + L * ((z0 + ez) % L))] = 0
        sl, sr = int(dec[row[0]]), int(dec[row[-1]])
        # from the left end: bonds js[0..h-1], from the right end js[h..2h-1]
        left, right = js[:h], js[h:]
        ref = (2 * sl * math.atanh((-1) ** h * np.prod(np.tanh(beta * left)))
               + 2 * sr * math.atanh((-1) ** h * np.prod(np.tanh(beta * right))))
        got = tn.site_score(L, J, dec, i, h, beta)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (trial, got, ref)
        # zero temperature: 2 s_f (-1)^k sgn(prod J) min |J| per side
        def side(s, jj):
            return 0 if np.any(jj == 0) else 2 * s * (-1) ** h * int(np.sign(np.prod(jj))) * int(np.abs(jj).min())
        assert tn.site_score(L, J, dec, i, h, tropical=True) == side(sl, left) + side(sr, right)


@pytest.mark.parametrize("tropical", [False, True])
def test_no_fixed_spin_is_exactly_even(tropical):
    L, h = 8, 1
    J = _rand_J(L, np.random.default_rng(11))
    dec = np.zeros(L ** 3, np.int8)
    for i in (0, 100, 511):
        assert tn.site_score(L, J, dec, i, h, 2.0, tropical) == 0


def _gauge(J, L, v):
    """Negate every coupling of site v (both stored copies)."""
    J = J.copy()
    x, y, z = v % L, (v // L) % L, v // (L * L)
    nb = [((x + 1) % L, y, z), ((x - 1) % L, y, z), (x, (y + 1) % L, z), (x, (y - 1) % L, z),
          (x, y, (z + 1) % L), (x, y, (z - 1) % L)]
    for d, (a, b, c) in enumerate(nb):
        u = a + L * (b + L * c)
        J[d, v] = -J[d, v]
        J[d ^ 1, u] = -J[d ^ 1, u]
    return J


@pytest.mark.parametrize("tropical", [False, True])
def test_gauge_invariance(tropical):
    L, h = 8, 2
    rng = np.random.default_rng(13)
    J = _rand_J(L, rng)
    i = 3 + L * (4 + L * 5)
    dec = rng.choice(np.array([-1, 0, 0, 1], np.int8), L ** 3).astype(np.int8)
    base = tn.site_score(L, J, dec, i, h, 2.0, tropical)
    assert base != 0
    free_v = next(v for v in (4 + L * (4 + L * 5), 3 + L * (5 + L * 5), 2 + L * (4 + L * 5)) if dec[v] == 0)
    fixed_v = next(v for v in (3 + L * (4 + L * 6), 3 + L * (3 + L * 5), 5 + L * (4 + L * 5),
                               1 + L * (4 + L * 5), 3 + L * (4 + L * 3)) if dec[v] != 0)
    tol = 0 if tropical else 1e-11 * abs(base)
    assert abs(tn.site_score(L, _gauge(J, L, free_v), dec, i, h, 2.0, tropical) - base) <= tol
    d2 = dec.copy()
    d2[fixed_v] = -d2[fixed_v]
    assert abs(tn.site_score(L, _gauge(J, L, fixed_v), d2, i, h, 2.0, tropical) - base) <= tol
    assert abs(tn.site_score(L, _gauge(J, L, i), dec, i, h, 2.0, tropical) + base) <= tol


def test_beta_limits():
    L, h = 8, 2
    rng = np.random.default_rng(17)
    J = _rand_J(L, rng)
    dec = rng.choice(np.array([-1, 0, 1], np.int8), L ** 3).astype(np.int8)
    for i in (9, 200, 333):
        assert tn.site_score(L, J, dec, i, h, 0.0) == 0.0
        d = tn.site_score(L, J, dec, i, h, tropical=True)
        beta = 400.0
        n_free = int(sum(1 for dz in range(-h, h + 1) for dy in range(-h, h + 1) for dx in range(-h, h + 1)
                         if dec[(i % L + dx) % L + L * ((((i // L) % L) + dy) % L + L * (((i // (L * L)) + dz) % L))] == 0))
        # |ln Z(s)/beta + E(s)| <= n_free ln 2 / beta on each side
        assert abs(tn.site_score(L, J, dec, i, h, beta) / beta - d) <= 2 * n_free * math.log(2) / beta + 1e-9


@pytest.mark.parametrize("order,h", [(1, 1), (0, 1)])
@pytest.mark.parametrize("tropical", [False, True])
def test_ferromagnet_decimates_to_ground_state(order, h, tropical):
    L = 6
    N = L ** 3
    J = np.full((6, N), -1, np.int8)
    dec, score = tn.tn_decimate(L, J, h, order, 2.0, tropical)
    assert np.all(dec == 1)
    assert oracle.energy(J, dec, (L, L, L)) == -3 * N
    # the first phase sees nothing fixed: an exact tie, broken to +1
    ph = np.array([tn.phase(order, L, h, i % L, (i // L) % L, i // (L * L)) for i in range(N)])
    assert np.all(score[ph == 0] == 0)
    assert np.all(score[ph > 0] > 0)


@pytest.mark.parametrize("order,h", [(1, 1), (0, 1)])
def test_antiferromagnet_decimates_to_neel_state(order, h):
    L = 6
    N = L ** 3
    J = np.full((6, N), 1, np.int8)
    dec, _ = tn.tn_decimate(L, J, h, order, 2.0)
    x, y, z = np.arange(N) % L, (np.arange(N) // L) % L, np.arange(N) // (L * L)
    neel = np.where((x + y + z) % 2 == 0, 1, -1)
    np.testing.assert_array_equal(dec, neel)
    assert oracle.energy(J, dec, (L, L, L)) == -3 * N


@pytest.mark.parametrize("tropical", [False, True])
def test_decisions_are_self_consistent_on_a_planted_instance(tropical):
    L, h = 6, 1
    J, _, egs = oracle.make_instance(L, 6, 12345)
    dec, score = tn.tn_decimate(L, J, h, 1, 2.0, tropical)
    assert set(np.unique(dec)) <= {-1, 1}
    assert oracle.energy(J, dec, (L, L, L)) >= egs
    ph = tn.phases(1, L, h)
    for i in range(0, L ** 3, 7):
        seen = tn.fixed_before(dec, ph, i)
        r = tn.site_score(L, J, seen, i, h, 2.0, tropical)
        assert r == score[i]
        assert dec[i] == (1 if r >= 0 else -1)
