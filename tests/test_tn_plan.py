"""Host checks of the tensor-network decimation planner (sg_tn_plan_*):
the elimination programs it exports, executed here in NumPy exactly as the
kernels execute them (table of 2^W entries, one pair update per eliminated
spin), give every site's score that the oracle's variable elimination
gives, for every distinct shape; plus the plan's bookkeeping and errors."""
import math

import numpy as np
import pytest

import paper_2501_17267_amd as sg
from oracle import tn

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _wrap(L, g, dx, dy, dz):
    x, y, z = g % L, (g // L) % L, g // (L * L)
    return (x + dx) % L + L * (((y + dy) % L) + L * ((z + dz) % L))


_DIRS = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def _execute(L, h, J, dec, site, shape, steps, beta, tropical, sc):
    """One table of one site: ln Z(sc) up to the fixed-fixed bonds, or the
    least energy, by the exported program."""
    W, ns, s0, cmask = (int(v) for v in shape)
    l = 2 * h + 1
    T = np.zeros(1 << W, np.int64) if tropical else np.ones(1 << W)
    log = 0.0
    idx = np.arange(1 << W, dtype=np.int64)
    for t in range(ns):
        lv, a, *codes = (int(v) for v in steps[s0 + t][:8])
        g = _wrap(L, site, lv % l - h, (lv // l) % l - h, lv // (l * l) - h)
        hc, act = 0, []
        for d, code in enumerate(codes):
            if code == -3:
                continue
            Jd = int(J[d, g])
            if code >= 0:
                act.append((Jd, code))
            elif code == -1:
                u = _wrap(L, g, *_DIRS[d])
                assert dec[u] != 0, "a fixed neighbour must be decimated"
                hc += Jd * int(dec[u])
            else:
                hc += Jd * sc
        I0 = idx[((idx >> a) & 1) == 0]
        I1 = I0 | (1 << a)
        hh = np.full(I0.shape, hc, np.int64)
        for Jd, b in act:
            hh += Jd * (1 - 2 * ((I0 >> b) & 1))
        if tropical:
            v = np.minimum(T[I0] + hh, T[I1] - hh)
        else:
            v = T[I0] * np.exp(-beta * hh) + T[I1] * np.exp(beta * hh)
            m = v.max()
            v = v / m
            log += math.log(m)
        T[I0] = v
        T[I1] = v
    assert np.all(T == T[0]), "the table must end constant"
    es = sum(int(J[d, site]) * int(dec[_wrap(L, site, *_DIRS[d])]) for d in range(6) if (cmask >> d) & 1) * sc
    return int(T[0]) + es if tropical else log + math.log(T[0]) - beta * es


def _execute_canonical(L, h, J, dec, site, shape, steps, beta, tropical, sc):
    """The same table by the workspace tier's rule: only canonical entries
    (free-slot bits 0) are read and written; each read pair (a = 0, 1, or
    one entry when slot a is new) writes every combination of the new slots."""
    W, ns, s0, cmask = (int(v) for v in shape)
    l = 2 * h + 1
    T = np.full(1 << W, -(1 << 40), np.int64) if tropical else np.full(1 << W, np.nan)
    T[0] = 0 if tropical else 1.0          # a fragment without free spins
    log = 0.0
    P = 0
    for t in range(ns):
        row = [int(v) for v in steps[s0 + t]]
        lv, a, codes = row[0], row[1], row[2:8]
        a_active, n_runs, n_base, newmask = row[8], row[9], row[10], row[11] & 0xFFFFFFFF
        starts = [(row[12 + r // 4] >> (8 * (r % 4))) & 0xFF for r in range(n_runs)]
        lens = [(row[14 + r // 4] >> (8 * (r % 4))) & 0xFF for r in range(n_runs)]
        assert a_active == ((P >> a) & 1) and sum(lens) == n_base
        assert (newmask & P) == 0 and not (newmask >> a) & 1
        base = P & ~(1 << a)
        assert sum(1 << (st + k) for st, ln in zip(starts, lens) for k in range(ln)) == base
        g = _wrap(L, site, lv % l - h, (lv // l) % l - h, lv // (l * l) - h)
        hc, act = 0, []
        for d, code in enumerate(codes):
            if code == -3:
                continue
            Jd = int(J[d, g])
            if code >= 0:
                assert ((P | newmask | (1 << a)) >> code) & 1
                act.append((Jd, code))
            elif code == -1:
                hc += Jd * int(dec[_wrap(L, g, *_DIRS[d])])
            else:
                hc += Jd * sc
        outs = {}
        for p in range(1 << n_base):
            I, used = 0, 0
            for st, ln in zip(starts, lens):
                I |= ((p >> used) & ((1 << ln) - 1)) << st
                used += ln
            if t == 0:
                t0 = t1 = 0 if tropical else 1.0
            else:
                t0 = T[I]
                t1 = T[I | (1 << a)] if a_active else t0
                assert (tropical and t0 != -(1 << 40)) or (not tropical and not np.isnan(t0))
            c = 0
            while True:
                O = I | c
                hh = hc + sum(Jd * (1 - 2 * ((O >> b) & 1)) for Jd, b in act)
                outs[O] = min(t0 + hh, t1 - hh) if tropical else t0 * math.exp(-beta * hh) + t1 * math.exp(beta * hh)
                c = (c - newmask) & newmask
                if c == 0:
                    break
        if not tropical:
            m = max(outs.values())
            log += math.log(m)
            outs = {k: v / m for k, v in outs.items()}
        for O, v in outs.items():
            T[O] = v
        P = (P | newmask | (1 << a)) & ~(1 << a)
    assert P == 0
    es = sum(int(J[d, site]) * int(dec[_wrap(L, site, *_DIRS[d])]) for d in range(6) if (cmask >> d) & 1) * sc
    return int(T[0]) + es if tropical else log + math.log(T[0]) - beta * es


def _terms(L, h, J, dec, site, row, sc):
    """Field terms of one step: the constant part and (J, slot) per active neighbour."""
    l = 2 * h + 1
    lv, codes = int(row[0]), [int(v) for v in row[2:8]]
    g = _wrap(L, site, lv % l - h, (lv // l) % l - h, lv // (l * l) - h)
    hc, act = 0, []
    for d, code in enumerate(codes):
        if code == -3:
            continue
        Jd = int(J[d, g])
        if code >= 0:
            act.append((Jd, code))
        elif code == -1:
            hc += Jd * int(dec[_wrap(L, g, *_DIRS[d])])
        else:
            hc += Jd * sc
    return hc, act


def _subsets(mask):
    c = 0
    while True:
        yield c
        c = (c - mask) & mask
        if c == 0:
            return


def _runs(row):
    n_runs = int(row[9])
    starts = [(int(row[12 + r // 4]) >> (8 * (r % 4))) & 0xFF for r in range(n_runs)]
    lens = [(int(row[14 + r // 4]) >> (8 * (r % 4))) & 0xFF for r in range(n_runs)]
    return starts, lens


def _deposit(p, starts, lens):
    I, used = 0, 0
    for st, ln in zip(starts, lens):
        I |= ((p >> used) & ((1 << ln) - 1)) << st
        used += ln
    return I


def _execute_rounds(L, h, J, dec, site, shape, steps, shape_rounds, rounds, sidx, beta, tropical, sc):
    """The table by the workspace tier's rule round by round, a fused round
    (steps t, t + 1) the way the step kernel runs it: per read assignment
    (canonical slots of t other than slot b of t + 1) the entries at a, b =
    0, 1 are read, step t's values kept, and only step t + 1's entries
    written; renormalised after each round.  Also checks that within a
    round no entry one assignment reads is written by another."""
    W, ns, s0, cmask = (int(v) for v in shape)
    r0, nr = (int(v) for v in shape_rounds[sidx])
    T = np.full(1 << W, -(1 << 40), np.int64) if tropical else np.full(1 << W, np.nan)
    T[0] = 0 if tropical else 1.0
    log = 0.0
    pair = ((lambda t0, t1, hh: min(t0 + hh, t1 - hh)) if tropical else
            (lambda t0, t1, hh: t0 * math.exp(-beta * hh) + t1 * math.exp(beta * hh)))
    field = lambda terms, idx: terms[0] + sum(Jd * (1 - 2 * ((idx >> b) & 1)) for Jd, b in terms[1])
    covered = 0
    for r in range(nr):
        t, fused, read_bits, bcode = (int(v) for v in rounds[r0 + r])
        assert t == covered, "rounds cover the steps in order"
        row = steps[s0 + t]
        a, a_active, n_base, nm = int(row[1]), int(row[8]), int(row[10]), int(row[11]) & 0xFFFFFFFF
        starts, lens = _runs(row)
        base = _deposit((1 << n_base) - 1, starts, lens)
        term0 = _terms(L, h, J, dec, site, row, sc)
        outs, reader, writer = {}, {}, {}
        if not fused:
            assert read_bits == n_base
            for p in range(1 << n_base):
                I = _deposit(p, starts, lens)
                t0 = t1 = 0 if tropical else 1.0
                if t > 0:
                    t0 = T[I]
                    t1 = T[I | (1 << a)] if a_active else t0
                for c in _subsets(nm):
                    outs[I | c] = pair(t0, t1, field(term0, I | c))
            covered += 1
        else:
            row1 = steps[s0 + t + 1]
            b, nm1 = int(row1[1]), int(row1[11]) & 0xFFFFFFFF
            mode, rank = bcode & 0xFF, bcode >> 8
            assert t + 2 < ns and b != a
            assert mode == (1 if (base >> b) & 1 else 2 if (nm >> b) & 1 else 0)
            assert int(row1[8]) == (mode != 0)
            kept = (1 << bin(nm).count("1")) * (2 if mode == 1 else 1)
            assert kept <= 8
            if mode == 1:
                assert rank == bin(base & ((1 << b) - 1)).count("1") and read_bits == n_base - 1
            else:
                assert read_bits == n_base
            term1 = _terms(L, h, J, dec, site, row1, sc)
            for p in range(1 << read_bits):
                q = p if mode != 1 else ((p >> rank) << (rank + 1)) | (p & ((1 << rank) - 1))
                I = _deposit(q, starts, lens)
                v0 = {}
                for ta in ((0, 1) if mode == 1 else (0,)):
                    Ib = I | (ta << b)
                    t0 = t1 = 0 if tropical else 1.0
                    if t > 0:
                        t0 = T[Ib]
                        reader.setdefault(Ib, set()).add(p)
                        if a_active:
                            t1 = T[Ib | (1 << a)]
                            reader.setdefault(Ib | (1 << a), set()).add(p)
                        else:
                            t1 = t0
                    for c in _subsets(nm):
                        v0[Ib | c] = pair(t0, t1, field(term0, Ib | c))
                assert len(v0) <= 8
                for c0 in _subsets(nm & ~(1 << b)):
                    B = I | c0
                    u0 = v0[B]
                    u1 = v0[B | (1 << b)] if mode else u0
                    for c1 in _subsets(nm1):
                        outs[B | c1] = pair(u0, u1, field(term1, B | c1))
                        writer[B | c1] = p
            for loc, ps in reader.items():
                assert loc not in writer or ps == {writer[loc]}, "an assignment writes what another reads"
            covered += 2
        if not tropical:
            m = max(outs.values())
            log += math.log(m)
            outs = {k: v / m for k, v in outs.items()}
        for O, v in outs.items():
            T[O] = v
    assert covered == ns
    es = sum(int(J[d, site]) * int(dec[_wrap(L, site, *_DIRS[d])]) for d in range(6) if (cmask >> d) & 1) * sc
    return int(T[0]) + es if tropical else log + math.log(T[0]) - beta * es


def _check_plan(L, h, order, n_sample=None, tropical=False, max_bits=None, seed=0):
    plan = sg.TnPlan(L, h, order)
    shapes, steps, items = plan.program()
    shape_rounds, rounds = plan.rounds()
    info = plan.info()
    assert info["n_shapes"] == len(shapes) and len(items) == L ** 3
    assert sorted(items[:, 0].tolist()) == list(range(L ** 3))
    rng = np.random.default_rng(seed)
    J, _, _ = sg.make_instance(L, 6, 777 + L + h)
    J = np.asarray(J).reshape(6, L ** 3)
    ph = tn.phases(order, L, h)
    # the items come phase by phase
    assert np.all(np.diff(ph[items[:, 0]]) >= 0)
    # one site of every shape (or all sites), each against the oracle
    first = {}
    for site, s in items:
        first.setdefault(int(s), int(site))
    sites = list(first.values())
    if max_bits is not None:
        sites = [first[s] for s in first if shapes[s][0] <= max_bits]
    if n_sample is not None and len(sites) > n_sample:
        sites = list(rng.choice(sites, n_sample, replace=False))
    shape_of = {int(site): int(s) for site, s in items}
    for site in sites:
        dec = np.where(ph < ph[site], rng.choice(np.array([-1, 1], np.int8), L ** 3), 0).astype(np.int8)
        zp = _execute(L, h, J, dec, site, shapes[shape_of[site]], steps, 2.0, tropical, 1)
        zm = _execute(L, h, J, dec, site, shapes[shape_of[site]], steps, 2.0, tropical, -1)
        got = (zm - zp) if tropical else (zp - zm)
        cp = _execute_canonical(L, h, J, dec, site, shapes[shape_of[site]], steps, 2.0, tropical, 1)
        cm = _execute_canonical(L, h, J, dec, site, shapes[shape_of[site]], steps, 2.0, tropical, -1)
        got_c = (cm - cp) if tropical else (cp - cm)
        ref = tn.site_score(L, J, dec, site, h, 2.0, tropical)
        sidx = shape_of[site]
        rp = _execute_rounds(L, h, J, dec, site, shapes[sidx], steps, shape_rounds, rounds, sidx, 2.0, tropical, 1)
        rm = _execute_rounds(L, h, J, dec, site, shapes[sidx], steps, shape_rounds, rounds, sidx, 2.0, tropical, -1)
        got_r = (rm - rp) if tropical else (rp - rm)
        if tropical:
            assert got_r == ref, (site, got_r, ref)
        else:
            assert abs(got_r - ref) <= 1e-9 * max(1.0, abs(ref)), (site, got_r, ref)
        if tropical:
            assert got_c == ref, (site, got_c, ref)
        else:
            assert abs(got_c - ref) <= 1e-9 * max(1.0, abs(ref)), (site, got_c, ref)
        if tropical:
            assert got == ref, (site, got, ref)
        else:
            assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (site, got, ref)
    return info


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("tropical", [False, True])
def test_every_shape_of_l3_plans_matches_the_oracle(order, tropical):
    _check_plan(6, 1, order, tropical=tropical)
    _check_plan(8, 1, order, tropical=tropical, seed=1)


@pytest.mark.parametrize("tropical", [False, True])
def test_l5_wavefront_light_shapes_match_the_oracle(tropical):
    info = _check_plan(12, 2, 1, n_sample=12, tropical=tropical, max_bits=12, seed=2)
    assert info["max_bits"] <= 26


def test_degenerate_single_site_fragments():
    # h = 0: every fragment is its own site, no bond, every table has 2^0 entries
    plan = sg.TnPlan(6, 0, 1)
    shapes, steps, items = plan.program()
    assert len(steps) == 0 and np.all(shapes[:, 0] == 0) and np.all(shapes[:, 1] == 0)
    assert plan.info()["pair_updates"] == 0


def test_plan_statistics():
    info = sg.TnPlan(20, 2, 1).info()
    assert info["n_phases"] == 58 and info["n_lds_sites"] + info["n_hbm_sites"] == 8000
    assert info["max_bits"] <= 22 and info["max_steps"] == 124
    # colour classes: phase 0 sees whole free cubes (124 free spins)
    info0 = sg.TnPlan(12, 2, 0).info()
    assert info0["n_phases"] == 27 and info0["max_steps"] == 124
    small = sg.TnPlan(20, 2, 1, 8).info()
    assert small["lds_max_bits"] == 8 and small["n_hbm_sites"] > info["n_hbm_sites"]


def test_workspace_sizes():
    plan = sg.TnPlan(12, 2, 1)
    lo, hi = plan.workspace_bytes(4, full=False), plan.workspace_bytes(4, full=True)
    assert 0 < lo <= hi
    # the least workspace holds the largest single table pair (2 x 2^22 doubles)
    assert lo >= 2 * 8 * (1 << plan.info()["max_bits"])


@pytest.mark.parametrize("L,h,order,bits", [(7, 1, 1, 0), (6, 3, 1, 0), (4, 2, 1, 0), (10, 2, 0, 0),
                                            (8, 1, 2, 0), (8, 1, 1, 14), (8, -1, 1, 0)])
def test_plan_argument_errors(L, h, order, bits):
    with pytest.raises(sg.SgError):
        sg.TnPlan(L, h, order, bits)


def test_workspace_step_bytes_accounting():
    # the algorithmic bytes the bench's TN roofline uses: linear in the
    # instances, half as many in the tropical form (4-byte entries), and for
    # one shape equal to a direct count over its exported program
    from paper_2501_17267_amd import tn_study
    one = tn_study.workspace_step_bytes(12, 2, 1, 8)
    assert one > 0 and tn_study.workspace_step_bytes(12, 2, 3, 8) == 3 * one
    assert 2 * tn_study.workspace_step_bytes(12, 2, 2, 4) == tn_study.workspace_step_bytes(12, 2, 2, 8)
    plan = sg.TnPlan(12, 2, 1)
    shapes, steps, items = plan.program()
    lb = plan.info()["lds_max_bits"]
    want = 0
    for _, s in items:
        W, ns, s0 = (int(v) for v in shapes[s][:3])
        if W <= lb:
            continue
        for t in range(ns):
            a_act, n_base, nm = int(steps[s0 + t][8]), int(steps[s0 + t][10]), int(steps[s0 + t][11]) & 0xFFFFFFFF
            reads = 0 if t == 0 else 1 + a_act
            want += 2 * (reads + 2 ** bin(nm).count("1")) * 2 ** n_base * 8
    assert tn_study.workspace_step_bytes(12, 2, 1, 8, fused=False) == want
    # fused rounds: the reads and writes of the round rule executed over
    # index sets (assignments x entries), for the four smallest workspace
    # shapes; then the total against the per-shape counts
    shape_rounds, rounds = plan.rounds()
    hbm_shapes = sorted({int(s) for _, s in items if shapes[s][0] > lb}, key=lambda s: int(shapes[s][0]))
    assert len(hbm_shapes) > 4
    for s in hbm_shapes[:4]:
        W, ns, s0 = (int(v) for v in shapes[s][:3])
        r0, nr = (int(v) for v in shape_rounds[s])
        want_f = 0
        for t, fz, read_bits, bcode in (tuple(int(v) for v in rounds[r0 + r]) for r in range(nr)):
            row = steps[s0 + t]
            starts, lens = _runs(row)
            a, a_act, nm = int(row[1]), int(row[8]), int(row[11]) & 0xFFFFFFFF
            reads, writes = set(), set()
            if not fz:
                for p in range(1 << int(row[10])):
                    I = _deposit(p, starts, lens)
                    if t > 0:
                        reads |= {I, I | (a_act << a)}
                    writes |= {I | c for c in _subsets(nm)}
            else:
                nxt = steps[s0 + t + 1]
                b, nm1, mode, rank = int(nxt[1]), int(nxt[11]) & 0xFFFFFFFF, bcode & 0xFF, bcode >> 8
                for p in range(1 << read_bits):
                    I = _deposit(((p >> rank) << (rank + 1)) | (p & ((1 << rank) - 1)) if mode == 1 else p,
                                 starts, lens)
                    for ta in ((0, 1) if mode == 1 else (0,)):
                        if t > 0:
                            reads |= {I | (ta << b), I | (ta << b) | (a_act << a)}
                    writes |= {I | c0 | c1 for c0 in _subsets(nm & ~(1 << b)) for c1 in _subsets(nm1)}
            want_f += len(reads) + len(writes)
        assert tn_study.shape_step_entries(shapes, steps, shape_rounds, rounds, s) == want_f
    per = {int(s): tn_study.shape_step_entries(shapes, steps, shape_rounds, rounds, int(s)) for s in hbm_shapes}
    assert one == sum(2 * per[int(s)] * 8 for _, s in items if int(s) in per) and one < 0.6 * want


@pytest.mark.parametrize("L,h,order", [(6, 1, 1), (8, 1, 0), (12, 2, 1), (12, 2, 0), (20, 2, 1)])
def test_tables_are_as_narrow_as_the_active_spins_allow(L, h, order):
    # every shape's table has exactly as many index bits as the most spins
    # active at once in its program (the slot assignment never widens it),
    # and the slots in use at a step are distinct bits below that width
    plan = sg.TnPlan(L, h, order)
    shapes, steps, _ = plan.program()
    for W, ns, s0, _ in (tuple(int(v) for v in sh) for sh in shapes):
        active, most = 0, 0
        for t in range(ns):
            row = steps[s0 + t]
            a, nm = int(row[1]), int(row[11]) & 0xFFFFFFFF
            now = active | nm | (1 << a)   # the slots in use while step t runs
            assert now >> W == 0
            most = max(most, bin(now).count("1"))
            active = now & ~(1 << a)
        assert most == W and active == 0
