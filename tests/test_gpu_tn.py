"""GPU parity of the tensor-network fragment decimation (sg_tn_decimate
through the C ABI) against the oracle (oracle/tn.py).

* l = 3: whole decimations against the oracle's, both phase orders, both
  forms (sum-product at beta = 2, tropical), in the LDS tier and with a
  forced low LDS limit in the workspace tier (with the least workspace, so
  that the workspace tables go in several passes), several instances per
  call.  Spins and energies identical, scores within 1e-9 (tropical: equal).
* l = 5 (the paper's fragment): every site's score from the LDS tier and
  from the workspace tier agree bit for bit (same arithmetic, same
  scaling); sampled sites of every table size the oracle finishes in
  seconds are checked against it from the decimated configuration.
* Exact ties: the uniform ferromagnet decimates to all +1 with the first
  phase's scores exactly 0; degenerate single-site fragments.
* Several instances per call (split into halves on two streams) equal
  one-instance calls bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from gpu_util import log
from oracle import tn

pytestmark = pytest.mark.gpu


def _instances(L, n, seed0):
    Js, egs = [], []
    for k in range(n):
        J, _, e = sg.make_instance(L, 6, seed0 + k)
        Js.append(np.asarray(J).reshape(6, L ** 3))
        egs.append(e)
    return Js, egs


def _run(plan, Js, beta, tropical, workspace=None):
    J = torch.from_numpy(np.stack(Js)).cuda()
    sp, en, sc = sg.tn_decimate(plan, J, beta, tropical, workspace=workspace)
    torch.cuda.synchronize()
    return sp.cpu().numpy(), en.cpu().numpy(), sc.cpu().numpy()


def _close(a, b):
    return abs(a - b) <= 1e-9 * max(1.0, abs(b))


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("tropical", [False, True])
@pytest.mark.parametrize("lds_bits", [0, 4, 1])
def test_l3_whole_decimation_equals_the_oracle(order, tropical, lds_bits):
    L, h, n = 6, 1, 3
    log(f"tn l=3 L={L} order={order} tropical={tropical} lds_bits={lds_bits}")
    plan = sg.TnPlan(L, h, order, lds_bits)
    if lds_bits:
        assert plan.info()["n_hbm_sites"] > 0
    Js, egs = _instances(L, n, 300 + order)
    ws = None
    if lds_bits:
        nbytes = plan.workspace_bytes(n, full=False)
        ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    sp, en, sc = _run(plan, Js, 2.0, tropical, ws)
    for b in range(n):
        ref, rsc = tn.tn_decimate(L, Js[b], h, order, 2.0, tropical)
        np.testing.assert_array_equal(sp[b], ref, err_msg=f"instance {b}")
        assert en[b] == oracle.energy(Js[b], ref, (L, L, L)) and en[b] >= egs[b]
        if tropical:
            np.testing.assert_array_equal(sc[b], rsc)
        else:
            assert all(_close(float(x), float(y)) for x, y in zip(sc[b], rsc))


def test_l3_larger_lattice_wavefront():
    L, h = 10, 1
    log(f"tn l=3 L={L}")
    plan = sg.TnPlan(L, h, 1)
    Js, egs = _instances(L, 1, 909)
    sp, en, sc = _run(plan, Js, 2.0, False)
    ref, rsc = tn.tn_decimate(L, Js[0], h, 1, 2.0)
    np.testing.assert_array_equal(sp[0], ref)
    assert en[0] == oracle.energy(Js[0], ref, (L, L, L))
    assert all(_close(float(x), float(y)) for x, y in zip(sc[0], rsc))


@pytest.mark.parametrize("tropical", [False, True])
def test_l5_tiers_agree_and_sites_match_the_oracle(tropical):
    L, h = 10, 2
    log(f"tn l=5 L={L} tropical={tropical}: LDS tier vs workspace tier")
    Js, egs = _instances(L, 2, 5151)
    p13 = sg.TnPlan(L, h, 1)
    p8 = sg.TnPlan(L, h, 1, 8)
    sp13, en13, sc13 = _run(p13, Js, 2.0, tropical)
    sp8, en8, sc8 = _run(p8, Js, 2.0, tropical)
    np.testing.assert_array_equal(sp13, sp8)
    np.testing.assert_array_equal(sc13, sc8)
    np.testing.assert_array_equal(en13, en8)
    shapes, _, items = p13.program()
    W = {int(site): int(shapes[s][0]) for site, s in items}
    ph = tn.phases(1, L, h)
    rng = np.random.default_rng(4)
    small = [i for i in range(L ** 3) if W[i] <= 13]
    picks = list(rng.choice(small, 10, replace=False))
    picks += [next(i for i in range(L ** 3) if W[i] == w) for w in (14, 17) if any(W[i] == w for i in range(L ** 3))]
    for b in range(2):
        assert en13[b] == oracle.energy(Js[b], sp13[b], (L, L, L)) and en13[b] >= egs[b]
        for i in picks[: (len(picks) if b == 0 else 4)]:
            log(f"  site {i} W={W[i]}")
            r = tn.site_score(L, Js[b], tn.fixed_before(sp13[b], ph, int(i)), int(i), h, 2.0, tropical)
            if tropical:
                assert sc13[b][i] == r
            else:
                assert _close(float(sc13[b][i]), r), (i, sc13[b][i], r)
            assert sp13[b][i] == (1 if r >= 0 else -1)


@pytest.mark.parametrize("tropical", [False, True])
def test_ferromagnet_ties_and_ground_state(tropical):
    L, h = 8, 2
    log(f"tn ferromagnet L={L} tropical={tropical}")
    N = L ** 3
    J = np.full((6, N), -1, np.int8)
    plan = sg.TnPlan(L, h, 1)
    sp, en, sc = _run(plan, [J], 2.0, tropical)
    assert np.all(sp[0] == 1) and en[0] == -3 * N
    ph = tn.phases(1, L, h)
    assert np.all(sc[0][ph == 0] == 0) and np.all(sc[0][ph > 0] > 0)


def test_single_site_fragments():
    L = 6
    plan = sg.TnPlan(L, 0, 1)
    Js, _ = _instances(L, 1, 12)
    sp, en, sc = _run(plan, Js, 2.0, False)
    assert np.all(sp == 1) and np.all(sc == 0)
    assert en[0] == oracle.energy(Js[0], sp[0], (L, L, L))


def test_full_size_run_is_sampled_against_the_oracle():
    # the measured configuration: L = 20, l = 5, beta = 2, wavefront order
    L, h = 20, 2
    log(f"tn full size L={L} l=5")
    plan = sg.TnPlan(L, h, 1)
    Js, egs = _instances(L, 2, 2020)
    sp, en, sc = _run(plan, Js, 2.0, False)
    assert set(np.unique(sp)) <= {-1, 1} and np.all(np.isfinite(sc))
    shapes, _, items = plan.program()
    W = {int(site): int(shapes[s][0]) for site, s in items}
    ph = tn.phases(1, L, h)
    rng = np.random.default_rng(20)
    for b in range(2):
        assert en[b] == oracle.energy(Js[b], sp[b], (L, L, L)) and en[b] >= egs[b]
        np.testing.assert_array_equal(sp[b], np.where(sc[b] >= 0, 1, -1))
        for i in rng.choice([i for i in range(L ** 3) if W[i] <= 13], 6, replace=False):
            r = tn.site_score(L, Js[b], tn.fixed_before(sp[b], ph, int(i)), int(i), h, 2.0)
            assert _close(float(sc[b][i]), r), (b, i, sc[b][i], r)
    log(f"  eps = {[(int(e) - g) / abs(g) for e, g in zip(en, egs)]}")


@pytest.mark.parametrize("tropical", [False, True])
def test_batch_halves_equal_single_instance_calls(tropical):
    # three instances in the workspace tier run as halves of one and two on
    # two streams; every instance equals its own one-instance call
    L, h = 10, 2
    log(f"tn batch halves L={L} tropical={tropical}")
    plan = sg.TnPlan(L, h, 1, 8)
    assert plan.info()["n_hbm_sites"] > 0
    Js, egs = _instances(L, 3, 7070)
    sp, en, sc = _run(plan, Js, 2.0, tropical)
    for b in range(3):
        sp1, en1, sc1 = _run(plan, [Js[b]], 2.0, tropical)
        np.testing.assert_array_equal(sp[b], sp1[0])
        np.testing.assert_array_equal(sc[b], sc1[0])
        assert en[b] == en1[0]


@pytest.mark.parametrize("beta", [8.0, 12.0])
def test_fused_pairs_and_single_steps_at_higher_beta(beta):
    # beta 8: fused pairs of steps; beta 12 (above SG_TN_FUSE_BETA_MAX):
    # every step its own round; in both tiers.  l = 3 against the oracle
    # with the workspace tier forced, l = 5 tiers bit-identical
    L, h = 6, 1
    log(f"tn l=3 L={L} beta={beta}")
    plan = sg.TnPlan(L, h, 1, 4)
    assert plan.info()["n_hbm_sites"] > 0
    Js, egs = _instances(L, 2, 1212)
    ws = torch.empty((plan.workspace_bytes(2, full=False) + 7) // 8, dtype=torch.float64, device="cuda")
    sp, en, sc = _run(plan, Js, beta, False, ws)
    for b in range(2):
        ref, rsc = tn.tn_decimate(L, Js[b], h, 1, beta, False)
        np.testing.assert_array_equal(sp[b], ref, err_msg=f"instance {b}")
        assert all(_close(float(x), float(y)) for x, y in zip(sc[b], rsc))
    L, h = 10, 2
    log(f"tn l=5 L={L} beta={beta}: LDS tier vs workspace tier")
    Js, _ = _instances(L, 1, 1213)
    sp13, en13, sc13 = _run(sg.TnPlan(L, h, 1), Js, beta, False)
    sp8, en8, sc8 = _run(sg.TnPlan(L, h, 1, 8), Js, beta, False)
    np.testing.assert_array_equal(sp13, sp8)
    np.testing.assert_array_equal(sc13, sc8)


def test_argument_errors():
    plan = sg.TnPlan(6, 1, 1)
    J = torch.zeros((1, 6, 216), dtype=torch.int8, device="cuda")
    with pytest.raises(sg.SgError):
        sg.tn_decimate(plan, J, beta=0.0)
    with pytest.raises(sg.SgError):
        sg.tn_decimate(plan, J, beta=25.0)
    with pytest.raises(sg.SgError):
        sg.tn_decimate(plan, J, beta=15.0)   # above the bound where no table overflows
    small = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sg.SgError):
        sg.tn_decimate(plan, J, beta=2.0, workspace=small)


def test_l5_colour_classes_whole_free_fragments():
    # colour classes at l = 5 (L = 6, period 3): the first class sees its whole
    # fragment free (the largest tables of any plan); its sites score exactly 0
    # and take +1; the tiers agree bit for bit; the ferromagnet decimates to
    # its ground state
    L, h = 6, 2
    log("tn l=5 colour classes L=6")
    plan, small = sg.TnPlan(L, h, 0), sg.TnPlan(L, h, 0, 8)
    assert plan.info()["max_bits"] >= 20
    Js, egs = _instances(L, 2, 606)
    sp, en, sc = _run(plan, Js, 2.0, False)
    sp8, en8, sc8 = _run(small, Js, 2.0, False)
    np.testing.assert_array_equal(sp, sp8)
    np.testing.assert_array_equal(sc, sc8)
    ph = tn.phases(0, L, h)
    for b in range(2):
        assert np.all(sc[b][ph == 0] == 0) and np.all(sp[b][ph == 0] == 1)
        assert en[b] == oracle.energy(Js[b], sp[b], (L, L, L)) and en[b] >= egs[b]
        np.testing.assert_array_equal(sp[b], np.where(sc[b] >= 0, 1, -1))
    J = np.full((6, L ** 3), -1, np.int8)
    spf, enf, _ = _run(plan, [J], 2.0, True)
    assert np.all(spf == 1) and enf[0] == -3 * L ** 3


def test_full_size_workspace_tier_sites_per_table_size():
    # the measured configuration (L = 20, l = 5, beta = 2, wavefront order):
    # one site of every workspace-tier table size from 2^14 up to 2^20 (the
    # largest the oracle contracts in about a minute) is compared with the
    # oracle's marginal, given the decimated spins of the earlier phases
    import concurrent.futures as cf
    L, h = 20, 2
    log(f"tn full size L={L} l=5: workspace-tier sites")
    plan = sg.TnPlan(L, h, 1)
    Js, egs = _instances(L, 1, 2020)
    sp, en, sc = _run(plan, Js, 2.0, False)
    shapes, _, items = plan.program()
    W = {int(site): int(shapes[s][0]) for site, s in items}
    ph = tn.phases(1, L, h)
    sizes = sorted({w for w in W.values() if 14 <= w <= 20})
    assert sizes[0] == 14 and sizes[-1] == 20
    picks = [next(i for i in range(L ** 3) if W[i] == w) for w in sizes]
    log(f"  table bits {sizes}, sites {picks}")

    def one(i):
        return i, tn.site_score(L, Js[0], tn.fixed_before(sp[0], ph, int(i)), int(i), h, 2.0)
    with cf.ThreadPoolExecutor(len(picks)) as ex:
        for i, r in ex.map(one, picks):
            log(f"  site {i} W={W[i]}: gpu {sc[0][i]!r} oracle {r!r}")
            assert _close(float(sc[0][i]), r), (i, W[i], sc[0][i], r)
            assert sp[0][i] == (1 if r >= 0 else -1)
