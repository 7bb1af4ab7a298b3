"""The no-allocation entry point sg_pt_run_split_static (split parallel
tempering whose mailbox lives in the library's fixed device array) against
the allocating sg_pt_run_split on the same inputs, through the C ABI: two
calls in a row, the second on a smaller input, bit for bit."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2501_17267_amd as sg
from gpu_util import dev_u32, instance, log

pytestmark = pytest.mark.gpu


def _static_call(inst, thr, thrx, n_runs, n_steps, seed, groups):
    T, K, M = int(thr.shape[0]), int(thr.shape[1]), int(thrx.shape[1])
    N = inst.L ** 3
    dev = inst.J.device
    sp = torch.empty((n_runs, T, N), dtype=torch.int8, device=dev)
    ps = torch.empty((n_runs, T), dtype=torch.int32, device=dev)
    en = torch.empty((n_runs, T), dtype=torch.int32, device=dev)
    tr = torch.empty((n_runs, n_steps), dtype=torch.int32, device=dev)
    sw = torch.zeros((n_runs, T - 1), dtype=torch.int32, device=dev)
    st = torch.full((1,), -7, dtype=torch.int32, device=dev)
    args = sg.sg_pt_args(n_runs=n_runs, run0=0, T=T, n_steps=n_steps, step0=0, K=K, M=M, init_random=1,
                         seed=seed)
    rc = sg.lib().sg_pt_run_split_static(ctypes.byref(inst.struct()), ctypes.byref(args), groups, 0,
                                         ctypes.c_void_p(thr.data_ptr()), ctypes.c_void_p(thrx.data_ptr()),
                                         ctypes.c_void_p(sp.data_ptr()), ctypes.c_void_p(en.data_ptr()),
                                         ctypes.c_void_p(ps.data_ptr()), ctypes.c_void_p(tr.data_ptr()),
                                         ctypes.c_void_p(sw.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, sg.lib().sg_last_error()
    return {"spins": sp, "energy": en, "pos": ps, "emin_trace": tr, "swap_acc": sw}, st


def _tables(T):
    beta = sg.make_schedule(1, 0.2, 3.0, T)
    M = sg.exchange_table_width(beta)
    return dev_u32(sg.make_thresholds(beta)), dev_u32(sg.make_exchange_thresholds(beta, M))


@pytest.mark.parametrize("first,second", [((12, 32, 16, 60, 2), (8, 16, 4, 25, 4)),
                                          ((10, 16, 9, 40, 8), (6, 8, 3, 17, 0))])
def test_static_split_pt_equals_allocating_form_twice(first, second):
    for k, (L, T, n_runs, n_steps, groups) in enumerate((first, second)):
        log(f"no-alloc split PT call {k}: L={L} T={T} runs={n_runs} steps={n_steps} groups={groups}")
        inst, Jo, go, egs = instance(L, 0x51A7 + 13 * L + k, 2)
        thr, thrx = _tables(T)
        seed = 0xC0FFEE + k
        got, st = _static_call(inst, thr, thrx, n_runs, n_steps, seed, groups)
        ref = sg.pt_run(inst, thr, thrx, n_runs, n_steps, seed, groups=groups, want_trace=True, want_swaps=True)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        if "workspace" in ref:
            assert int(ref["workspace"].view(torch.int32)[0].item()) == 0
        for key in ("spins", "energy", "pos", "emin_trace", "swap_acc"):
            assert torch.equal(got[key], ref[key]), (k, key)
