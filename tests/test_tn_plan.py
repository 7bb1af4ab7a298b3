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


def _check_plan(L, h, order, n_sample=None, tropical=False, max_bits=None, seed=0):
    plan = sg.TnPlan(L, h, order)
    shapes, steps, items = plan.program()
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
    assert one == want
