"""GPU parity of the fragment decimation (sg_fragment_decimate through the C
ABI) against the oracle: every decimated configuration and its energy,
bit for bit, for both phase orders, single-spin and block cores, fragment
edges from 1 to the largest, several anneals per fragment and several runs."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from gpu_util import dev_u32, instance, log

pytestmark = pytest.mark.gpu
K = 24


def _compare(L, core, halo, R, order, S, n_runs=2, run0=0, seed=0x51A7, beta=(0.1, 3.0)):
    log(f"fragment parity L={L} c={core} h={halo} R={R} order={order} S={S} runs={n_runs}")
    inst, Jo, go, egs = instance(L, 4000 + L + 10 * core + halo, 1)
    thr = sg.make_thresholds(sg.make_schedule(0, beta[0], beta[1], S), K)
    sp, en = sg.fragment_decimate(inst, dev_u32(thr), core, halo, R, order, n_runs, seed, run0=run0)
    torch.cuda.synchronize()
    sp, en = sp.cpu().numpy(), en.cpu().numpy()
    for i in range(n_runs):
        ref = oracle.frag_decimate(L, Jo, core, halo, R, seed, run0 + i, thr, order=order)
        np.testing.assert_array_equal(sp[i], ref, err_msg=f"run {i}")
        assert en[i] == oracle.energy(Jo, ref, (L, L, L))
        assert en[i] >= egs
    return sp, en


@pytest.mark.parametrize("order", [0, 1])
def test_single_spin_fragments_of_edge_five(order):
    # the paper's fragment edge l = 5 with one decimated spin per fragment
    _compare(12, 1, 2, 4, order, 8)


@pytest.mark.parametrize("L,core,halo,R,order", [
    (8, 1, 1, 2, 0), (8, 1, 1, 3, 1),          # l = 3
    (12, 3, 1, 8, 0), (12, 3, 1, 8, 1),        # block cores, l = 5
    (12, 2, 2, 16, 1),                         # the most anneals per fragment
    (10, 5, 2, 2, 1),                          # the largest fragment, l = 9
    (16, 2, 1, 5, 0), (16, 4, 2, 1, 1),        # one anneal per fragment
    (6, 1, 0, 3, 0), (6, 1, 0, 3, 1),          # l = 1: no bond inside a fragment
])
def test_fragment_shapes_bit_exact(L, core, halo, R, order):
    _compare(L, core, halo, R, order, 6, n_runs=3, run0=11)


def test_zero_temperature_and_long_anneal():
    # beta = infinity (all thresholds zero) and a longer schedule
    L, S = 12, 30
    inst, Jo, go, egs = instance(L, 77, 2)
    thr = np.zeros((5, K), np.uint32)
    sp, en = sg.fragment_decimate(inst, dev_u32(thr), 1, 2, 2, 1, 1, 9)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sp.cpu().numpy()[0], oracle.frag_decimate(L, Jo, 1, 2, 2, 9, 0, thr, order=1))
    _compare(L, 3, 1, 8, 1, S, n_runs=1)


def test_full_size_run_is_sampled_against_the_oracle():
    # the measured configuration (l = 5 single-spin fragments, 8 anneals of
    # 100 sweeps each) at L = 16, run 0 of several against the oracle, the
    # energies of all of them
    L = 16
    inst, Jo, go, egs = instance(L, 9016, 3)
    thr = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 100), K)
    log("fragment full size L=16 c=1 h=2 R=8 S=100")
    sp, en = sg.fragment_decimate(inst, dev_u32(thr), 1, 2, 8, 1, 4, 0xF00D)
    torch.cuda.synchronize()
    sp, en = sp.cpu().numpy(), en.cpu().numpy()
    ref = oracle.frag_decimate(L, Jo, 1, 2, 8, 0xF00D, 0, thr, order=1)
    np.testing.assert_array_equal(sp[0], ref)
    assert en[0] == oracle.energy(Jo, ref, (L, L, L))
    for i in range(4):
        assert en[i] == oracle.energy(Jo, sp[i], (L, L, L))
