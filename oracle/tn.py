"""Oracle for the tensor-network fragment decimation (App. A-C).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
library never loads it and shares no code with it.  Plain NumPy, float64.

What it computes (App. C and its bootstrapping figure; Sec. I):

* Spins are decimated one at a time, phase by phase.  The fragment of site i
  is the l^3 cube (l = 2h + 1) centred on i, with periodic wrap.  Only bonds
  whose two ends both lie in the cube belong to it.
* A fragment site decimated in an earlier phase is fixed at its value.  Every
  other fragment site is free (a site of the same phase counts as free: all
  sites of a phase see the state at the start of the phase).
* The marginal of i conditional on the fixed spins is the exact contraction
  of the fragment's Boltzmann-weight network at inverse temperature beta:
  Z(s_i) = sum over the free spins other than i of exp(-beta E_frag), with
  E_frag = sum of J_ab s_a s_b over the fragment's bonds (Eq. 1's sign).
  The spin takes its most probable value: +1 when ln Z(+1) >= ln Z(-1).
* The tropical variant (Sec. III) replaces (sum, product) by (min, +): the
  least fragment energy with s_i = +1 and with s_i = -1; +1 when
  E(+1) <= E(-1).

The contraction here is textbook variable elimination (bucket elimination)
in increasing local-index order: multiply the factors that hold a variable,
sum (or minimise) it out, repeat.  The sum-product form works on logarithms
(-beta E per factor, log-sum-exp to sum a variable out), so no table can
overflow or underflow at any beta.

Phase orders (single-spin cores): 0 = colour classes
(x mod P) + P((y mod P) + P(z mod P)) with P = 1 + h, so that no two sites
of one class share a fragment; 1 = diagonal wavefront x + y + z.
"""
from __future__ import annotations

import math

import numpy as np

# directions of J[6][N]: +x, -x, +y, -y, +z, -z
_FWD = ((0, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1)))


def n_phases(order: int, L: int, h: int) -> int:
    P = 1 + h
    return P ** 3 if order == 0 else 3 * (L - 1) + 1


def phase(order: int, L: int, h: int, x: int, y: int, z: int) -> int:
    P = 1 + h
    if order == 0:
        return (x % P) + P * ((y % P) + P * (z % P))
    return x + y + z


def params_ok(L: int, h: int, order: int) -> bool:
    l = 2 * h + 1
    if L < 4 or L % 2 or h < 0 or l >= L or order not in (0, 1):
        return False
    return order == 1 or L % (1 + h) == 0


def fragment(L: int, J: np.ndarray, dec: np.ndarray, i: int, h: int):
    """The fragment of site i: (global index per local site, bonds
    [(a, b, J)] between local sites, fixed values per local site, 0 = free).
    Local site j = lx + l (ly + l lz), lx = dx + h."""
    l = 2 * h + 1
    x0, y0, z0 = i % L, (i // L) % L, i // (L * L)
    n3 = l ** 3
    g = np.empty(n3, np.int64)
    for lz in range(l):
        for ly in range(l):
            for lx in range(l):
                gx, gy, gz = (x0 + lx - h) % L, (y0 + ly - h) % L, (z0 + lz - h) % L
                g[lx + l * (ly + l * lz)] = gx + L * (gy + L * gz)
    bonds = []
    for lz in range(l):
        for ly in range(l):
            for lx in range(l):
                a = lx + l * (ly + l * lz)
                for d, (ex, ey, ez) in _FWD:
                    mx, my, mz = lx + ex, ly + ey, lz + ez
                    if mx < l and my < l and mz < l:
                        bonds.append((a, mx + l * (my + l * mz), int(J[d, g[a]])))
    fixed = np.asarray(dec, np.int8)[g].astype(np.int64)
    return g, bonds, fixed


# ---- variable elimination ---------------------------------------------------

def _expand(vars_, arr, union):
    """arr over sorted vars_ seen as an array over the sorted union."""
    shape = [2 if v in vars_ else 1 for v in union]
    return arr.reshape(shape)


def _logsumexp(a, axis):
    m = a.max(axis=axis)
    return m + np.log(np.exp(a - np.expand_dims(m, axis)).sum(axis=axis))


def _eliminate(factors, order, tropical):
    """factors: list of (sorted var tuple, array over them): energies
    (tropical) or log-weights -beta E.  Eliminate the variables of `order`
    one by one: add the factors that hold the variable, then take the
    minimum (tropical) or log-sum-exp over it.  Returns the sum of the
    scalars left: the least energy, or ln Z."""
    factors = list(factors)
    for v in order:
        hold = [f for f in factors if v in f[0]]
        factors = [f for f in factors if v not in f[0]]
        union = tuple(sorted(set().union(*[f[0] for f in hold])))
        acc = np.zeros([1] * len(union), np.int64 if tropical else np.float64)
        for vs, arr in hold:
            acc = acc + _expand(vs, arr, union)
        acc = np.broadcast_to(acc, [2] * len(union))
        ax = union.index(v)
        out = acc.min(axis=ax) if tropical else _logsumexp(acc, ax)
        factors.append((tuple(u for u in union if u != v), out))
    if tropical:
        return int(sum(int(arr) for _, arr in factors))
    return float(sum(float(arr) for _, arr in factors))


def site_value(L, J, dec, i, h, beta, tropical, s_centre):
    """ln Z(s_centre) (or the least fragment energy with the centre at
    s_centre) of the fragment of i, conditional on the nonzero entries of
    dec inside it (the centre's own entry is ignored)."""
    g, bonds, fixed = fragment(L, J, dec, i, h)
    l = 2 * h + 1
    c = (l ** 3) // 2                       # local index of the centre
    val = fixed.copy()
    val[c] = s_centre
    free = [j for j in range(l ** 3) if val[j] == 0]
    s = np.array([1, -1], np.int64)
    factors = []
    const = 0                               # energy of bonds between fixed sites
    for a, b, Jab in bonds:
        fa, fb = val[a] == 0, val[b] == 0
        if fa and fb:
            e = Jab * np.outer(s, s)
            vs = (a, b) if a < b else (b, a)
            arr = e if a < b else e.T
        elif fa or fb:
            v, other = (a, b) if fa else (b, a)
            vs, arr = (v,), Jab * s * int(val[other])
        else:
            const += Jab * int(val[a]) * int(val[b])
            continue
        factors.append((vs, arr.astype(np.int64) if tropical else -beta * arr.astype(np.float64)))
    # a free site with no bond in the fragment still counts its two values
    touched = set(v for f in factors for v in f[0])
    for v in free:
        if v not in touched:
            factors.append(((v,), np.zeros(2, np.int64 if tropical else np.float64)))
    r = _eliminate(factors, sorted(free), tropical)
    return r + const if tropical else r - beta * const


def site_score(L, J, dec, i, h, beta=2.0, tropical=False):
    """The decision statistic of site i given the fixed spins in dec:
    ln Z(+1) - ln Z(-1), or E(-1) - E(+1) in the tropical variant (an int);
    the site takes +1 when it is >= 0."""
    zp = site_value(L, J, dec, i, h, beta, tropical, 1)
    zm = site_value(L, J, dec, i, h, beta, tropical, -1)
    return (zm - zp) if tropical else (zp - zm)


def tn_decimate(L, J, h, order=1, beta=2.0, tropical=False):
    """Decimate every site, phase by phase.  Returns (dec int8 [N], score
    [N]: each site's decision statistic, float64)."""
    if not params_ok(L, h, order):
        raise ValueError(f"tn_decimate: L={L} h={h} order={order}")
    J = np.asarray(J, np.int8).reshape(6, L ** 3)
    N = L ** 3
    dec = np.zeros(N, np.int8)
    score = np.zeros(N, np.float64)
    ph = phases(order, L, h)
    for q in range(n_phases(order, L, h)):
        snap = dec.copy()
        for i in np.nonzero(ph == q)[0]:
            r = site_score(L, J, snap, int(i), h, beta, tropical)
            score[i] = r
            dec[i] = 1 if r >= 0 else -1
    return dec, score


def phases(order: int, L: int, h: int) -> np.ndarray:
    """Phase of every site, [N]."""
    i = np.arange(L ** 3)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    P = 1 + h
    if order == 0:
        return (x % P) + P * ((y % P) + P * (z % P))
    return x + y + z


def fixed_before(dec, ph, i):
    """dec restricted to the sites of phases before site i's (what site i's
    fragment saw), from a finished decimation; ph = phases(...)."""
    return np.where(ph < ph[i], np.asarray(dec, np.int8), 0).astype(np.int8)
