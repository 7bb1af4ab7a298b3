"""Every launch shape (variant) of the annealing kernel must give the same
chains bit for bit; the autotuner checks this itself and must select a
variant."""
import numpy as np
import pytest
import torch

import paper_2501_17267_amd as sg
from gpu_util import dev_u32, instance, log, oracle_sa_parallel

pytestmark = pytest.mark.gpu
K = 24


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24, 26, 28, 30, 32, 64])
def test_every_variant_bit_exact(L):
    n_rep = 21 if L <= 32 else 3  # ragged against every replicas-per-group choice
    S = 5 if L <= 32 else 2
    inst, Jo, go, egs = instance(L, 0xA5A5 + L, 11)
    thr_h = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S), K)
    thr = dev_u32(thr_h)
    reps = [0, 7, 20] if n_rep == 21 else [0, 2]
    ref = oracle_sa_parallel(L, Jo, 0x77, 11, thr_h, reps, want_emin=True)
    for v, info in enumerate(sg.sa_variants(L)):
        log(f"variant L={L} v={v} {info}")
        for emin in (False, True):
            sp, en, em = sg.sa_anneal_variant(inst, thr, n_rep, 0x77, v, want_emin=emin)
            torch.cuda.synchronize()
            sp, en = sp.cpu().numpy(), en.cpu().numpy()
            for r in reps:
                np.testing.assert_array_equal(sp[r], ref[r][0], err_msg=f"L={L} v={v} r={r}")
                assert en[r] == ref[r][1]
                if emin:
                    assert em.cpu().numpy()[r] == ref[r][2]


@pytest.mark.parametrize("L", [8, 16])
def test_autotune_selects_an_identical_variant(L):
    before = sg.selected_variant(L)
    res = sg.autotune(L, n_rep=2048, n_sweeps=8, repeats=2)
    log(f"autotune L={L}: {res}")
    assert all(r["identical"] for r in res["results"])
    assert 0 <= res["selected"] < len(sg.sa_variants(L))
    assert sg.selected_variant(L) == res["selected"]
    best = min(res["results"], key=lambda r: r["ms"])
    assert res["results"][res["selected"]]["ms"] == best["ms"]
    sg.select_variant(L, before)
