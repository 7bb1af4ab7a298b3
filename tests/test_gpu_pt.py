"""GPU parity of parallel tempering (pt_run through the C ABI) against the
oracle: bit-exact spins, energies, ladder positions, per-step minimum
energies and exchange counts."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from paper_2501_17267_amd import workloads as wl
from gpu_util import CORES, dev_u32, instance, log

pytestmark = pytest.mark.gpu
K = 24


def _compare(L, T, n_runs, n_steps, seed, run0=0, step0=0, sample=None, b=(0.2, 3.0)):
    log(f"PT parity L={L} T={T} runs={n_runs} steps={n_steps} seed={seed:#x}")
    inst, Jo, go, egs = instance(L, seed + L, 0)
    beta = sg.make_schedule(1, b[0], b[1], T)
    thr = sg.make_thresholds(beta, K)
    M = sg.exchange_table_width(beta)
    thrx = sg.make_exchange_thresholds(beta, M)
    out = sg.pt_run(inst, dev_u32(thr), dev_u32(thrx), n_runs, n_steps, seed, run0=run0, step0=step0,
                    want_trace=True, want_swaps=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    runs = list(range(n_runs)) if sample is None else sample

    def one(r):
        return r, oracle.pt_run(L, Jo, seed, run0 + r, thr, thrx, n_steps, step0=step0,
                                want_trace=True, want_swaps=True)
    with cf.ThreadPoolExecutor(CORES) as ex:
        ref = dict(ex.map(one, runs))
    for r in runs:
        np.testing.assert_array_equal(got["spins"][r], ref[r]["spins"], err_msg=f"run {r}")
        np.testing.assert_array_equal(got["energy"][r], ref[r]["energy"])
        np.testing.assert_array_equal(got["pos"][r], ref[r]["pos"])
        np.testing.assert_array_equal(got["emin_trace"][r], ref[r]["emin_trace"])
        np.testing.assert_array_equal(got["swap_acc"][r].astype(np.uint32), ref[r]["swap_acc"])
    return got


@pytest.mark.parametrize("L,T", [(4, 2), (4, 5), (6, 8), (8, 16), (10, 7), (12, 32), (14, 12), (16, 8)])
def test_pt_bit_exact(L, T):
    _compare(L, T, 3, 12, 0x5EED + T)


def test_pt_offsets_and_resume():
    L, T = 8, 6
    inst, Jo, go, egs = instance(L, 17, 0)
    beta = sg.make_schedule(1, 0.2, 3.0, T)
    thr = dev_u32(sg.make_thresholds(beta, K))
    M = sg.exchange_table_width(beta)
    thrx = dev_u32(sg.make_exchange_thresholds(beta, M))
    full = sg.pt_run(inst, thr, thrx, 4, 20, 7, run0=9)
    a = sg.pt_run(inst, thr, thrx, 4, 8, 7, run0=9)
    b = sg.pt_run(inst, thr, thrx, 4, 12, 7, run0=9, step0=8, spins=a["spins"].clone(), pos=a["pos"].clone())
    torch.cuda.synchronize()
    for k in ("spins", "energy", "pos"):
        assert torch.equal(full[k], b[k]), k


def test_pt_workload_full_size_sampled_run():
    # the PT workload at full size (128 runs x 2000 steps, 32 temperatures,
    # L = 12); runs are independent, run 0 and run 127 are re-run by the oracle
    w = wl.pt()
    log("PT workload full size", w.n_runs, w.n_steps)
    inst, Jo, go, egs = instance(w.instance.L, w.instance.seed, 0)
    beta = sg.make_schedule(1, w.beta0, w.beta1, w.T)
    thr = sg.make_thresholds(beta, K)
    M = sg.exchange_table_width(beta)
    thrx = sg.make_exchange_thresholds(beta, M)
    out = sg.pt_run(inst, dev_u32(thr), dev_u32(thrx), w.n_runs, w.n_steps, w.seed, want_trace=True,
                    want_swaps=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    for r in range(w.n_runs):
        assert sorted(got["pos"][r]) == list(range(w.T))
    with cf.ThreadPoolExecutor(2) as ex:
        refs = list(ex.map(lambda r: (r, oracle.pt_run(w.instance.L, Jo, w.seed, r, thr, thrx, w.n_steps,
                                                       want_trace=True, want_swaps=True)), [0, 127]))
    for r, ref in refs:
        np.testing.assert_array_equal(got["spins"][r], ref["spins"])
        np.testing.assert_array_equal(got["energy"][r], ref["energy"])
        np.testing.assert_array_equal(got["pos"][r], ref["pos"])
        np.testing.assert_array_equal(got["emin_trace"][r], ref["emin_trace"])
        np.testing.assert_array_equal(got["swap_acc"][r].astype(np.uint32), ref["swap_acc"])
