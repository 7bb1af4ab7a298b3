"""The App. D harness end to end on the device, at reduced sizes: SA range
tuning over the full grid, PT ladder tuning over the full grid, TT-eps of
SA and of PT with cluster moves, and the alpha fits; the per-instance mean
gaps it decides on come from epsilon_stats and are checked here against the
oracle's statistics of the same energies."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from paper_2501_17267_amd import tuning as tu
from gpu_util import log

pytestmark = pytest.mark.gpu


def test_appd_harness_small():
    sa = tu.sa_tune(torch, L=6, n_inst=2, n_runs=4, s_max=64, per_octave=2, log=log)
    assert set(sa["targets"]) == {"0.03", "0.04", "0.05"}
    for t, v in sa["targets"].items():
        s = v["schedule"]
        if s is not None:
            assert 0.3 <= s["beta_min"] <= 3.3 and 3.0 <= s["beta_max"] <= 27.0
    pt = tu.pt_tune(torch, L=4, n_inst=1, n_runs=4, log=log)
    lad = {float(t): (v["ladder"]["T"], v["ladder"]["beta_min"], v["ladder"]["beta_max"])
           for t, v in pt["targets"].items() if v["ladder"]}
    assert lad and all(T in (2, 3, 4) for T, _, _ in lad.values())
    sched = {0.05: (1.0, 6.0)}
    a = tu.sa_alpha(torch, sched, sizes=(6, 8, 10), n_inst=2, n_trials=3, s_max=512, log=log)
    e = a["per_L"]["8"]["targets"]["0.05"]
    if not e["censored"]:
        assert e["plain_ms"] > 0 and e["batched_ms_per_trial"] > 0
    p = tu.pticm_alpha(torch, {0.05: lad[min(lad)]}, sizes=(4, 6), n_inst=2, n_trials=2, n_steps=200, log=log)
    assert set(p["per_L"]) == {"4", "6"}
    log(f"alpha table {tu.alpha_table({'sa_alpha': a, 'pticm_alpha': p})}")


def test_best_so_far_gap_matches_oracle_statistics():
    # the PT criterion's mean gap of the best-so-far energies (epsilon_stats
    # over cummin of the per-step minima) against the oracle's statistics of
    # the same energies
    inst = sg.Instance.generate(6, 4242, chain=0)
    beta = sg.make_schedule(1, 0.3, 4.0, 3)
    thr = sg.to_device_u32(sg.make_thresholds(beta))
    thrx = sg.to_device_u32(sg.make_exchange_thresholds(beta, sg.exchange_table_width(beta)))
    out = sg.pt_run(inst, thr, thrx, 7, 15, 99, want_trace=True)
    m = tu._best_so_far_eps(torch, out["emin_trace"], inst.E_gs)
    tr = out["emin_trace"].cpu().numpy()
    best = np.minimum.accumulate(tr, axis=1).T.copy()
    ref = oracle.eps_stats(best.astype(np.int32), [inst.E_gs] * best.shape[0])
    n = best.shape[1]
    ref_m = (ref["sum"] - n * inst.E_gs) / (n * abs(inst.E_gs))
    np.testing.assert_array_equal(m, ref_m)
