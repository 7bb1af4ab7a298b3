"""GPU parity of parallel tempering with isoenergetic cluster moves
(sg_pticm_run through the C ABI) against the oracle: final spins, energies,
slot positions, the per-step best energy, exchange counts and the sites
flipped by the cluster moves, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from gpu_util import dev_u32, instance, log

pytestmark = pytest.mark.gpu
K = 24


def _tables(T, beta_max=3.0):
    beta = sg.make_schedule(1, 0.2, beta_max, T)
    M = sg.exchange_table_width(beta)
    return sg.make_thresholds(beta, K), sg.make_exchange_thresholds(beta, M)


def _compare(L, T, icm_from, n_runs, n_steps, seed=0x1C3, run0=0):
    log(f"PT+ICM parity L={L} T={T} icm_from={icm_from} runs={n_runs} steps={n_steps}")
    inst, Jo, go, egs = instance(L, 6000 + L + T, 2)
    thr, thrx = _tables(T)
    out = sg.pticm_run(inst, dev_u32(thr), dev_u32(thrx), n_runs, n_steps, seed, icm_from=icm_from, run0=run0,
                       want_trace=True, want_swaps=True, want_icm=True)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    for r in range(n_runs):
        ref = oracle.pticm_run(L, Jo, seed, run0 + r, thr, thrx, n_steps, icm_from=icm_from, want_trace=True,
                               want_swaps=True, want_icm=True)
        np.testing.assert_array_equal(g["spins"][r], ref["spins"], err_msg=f"spins run {r}")
        np.testing.assert_array_equal(g["energy"][r], ref["energy"])
        np.testing.assert_array_equal(g["pos"][r], ref["pos"])
        np.testing.assert_array_equal(g["emin_trace"][r], ref["emin_trace"])
        np.testing.assert_array_equal(g["swap_acc"][r], ref["swap_acc"].astype(np.int32))
        np.testing.assert_array_equal(g["icm_flipped"][r], ref["icm_flipped"])
    return g


@pytest.mark.parametrize("L,T,icm_from", [(4, 2, 0), (6, 4, 0), (8, 8, 2), (10, 5, 1), (12, 8, 0), (12, 32, 16),
                                          (14, 4, 0), (16, 6, 3)])
def test_pticm_bit_exact(L, T, icm_from):
    g = _compare(L, T, icm_from, 2, 8)
    if icm_from < T:
        assert g["icm_flipped"].sum() > 0


def test_pticm_without_moves_copy_zero_is_pt():
    L, T = 8, 6
    inst, Jo, go, egs = instance(L, 66, 1)
    thr, thrx = _tables(T)
    a = sg.pticm_run(inst, dev_u32(thr), dev_u32(thrx), 3, 12, 0xAB, icm_from=T, want_swaps=True)
    p = sg.pt_run(inst, dev_u32(thr), dev_u32(thrx), 3, 12, 0xAB, want_swaps=True)
    torch.cuda.synchronize()
    assert torch.equal(a["spins"][:, :T], p["spins"])
    assert torch.equal(a["energy"][:, :T], p["energy"])
    assert torch.equal(a["pos"][:, :T], p["pos"])
    assert torch.equal(a["swap_acc"][:, :T - 1], p["swap_acc"])


def test_pticm_resume_equals_uninterrupted():
    L, T = 10, 6
    inst, Jo, go, egs = instance(L, 67, 3)
    thr, thrx = _tables(T)
    full = sg.pticm_run(inst, dev_u32(thr), dev_u32(thrx), 2, 17, 0xCD, icm_from=2)
    a = sg.pticm_run(inst, dev_u32(thr), dev_u32(thrx), 2, 10, 0xCD, icm_from=2)
    b = sg.pticm_run(inst, dev_u32(thr), dev_u32(thrx), 2, 7, 0xCD, icm_from=2, step0=10,
                     spins=a["spins"].clone(), pos=a["pos"].clone())
    torch.cuda.synchronize()
    assert torch.equal(full["spins"], b["spins"]) and torch.equal(full["energy"], b["energy"])
    assert torch.equal(full["pos"], b["pos"])
