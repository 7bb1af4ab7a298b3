"""GPU parity of parallel tempering spread over several work groups per run
(sg_pt_run_split through the C ABI): bit-exact against the oracle (spins,
energies, ladder positions, per-step minimum energies, exchange counts) for
every group count, ragged run counts (not a multiple of the eight runs a
launch chunk holds), explicit wave counts and resumed runs; at the PT
workload's full size it equals the one-group pt_run on every run and the
oracle on a sampled run; it runs ladders whose walkers do not fit one work
group's LDS (L = 16, 32 walkers); captured in a hipGraph, every replay equals
the eager call.  Every call's status word must read 0 (no group gave up
waiting on another)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from paper_2501_17267_amd import workloads as wl
from gpu_util import dev_u32, instance, log

pytestmark = pytest.mark.gpu
K = 24


def _ladder(T, b=(0.2, 3.0)):
    beta = sg.make_schedule(1, b[0], b[1], T)
    thr = sg.make_thresholds(beta, K)
    M = sg.exchange_table_width(beta)
    return thr, sg.make_exchange_thresholds(beta, M)


def _status(out):
    return int(out["workspace"].view(torch.int32)[0].item())


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if k != "workspace" and v is not None}


def _check_oracle(L, Jo, got, seed, runs, thr, thrx, n_steps, run0=0, step0=0, spins=None, pos=None):
    for r in runs:
        ref = oracle.pt_run(L, Jo, seed, run0 + r, thr, thrx, n_steps, step0=step0,
                            spins=None if spins is None else spins[r], pos=None if pos is None else pos[r],
                            want_trace=True, want_swaps=True)
        np.testing.assert_array_equal(got["spins"][r], ref["spins"], err_msg=f"run {r}")
        np.testing.assert_array_equal(got["energy"][r], ref["energy"])
        np.testing.assert_array_equal(got["pos"][r], ref["pos"])
        np.testing.assert_array_equal(got["emin_trace"][r], ref["emin_trace"])
        np.testing.assert_array_equal(got["swap_acc"][r].astype(np.uint32), ref["swap_acc"])


@pytest.mark.parametrize("L,T,groups", [(4, 4, 2), (6, 8, 4), (8, 16, 8), (10, 6, 2), (12, 32, 2), (12, 32, 4),
                                        (14, 12, 4), (16, 8, 2), (12, 32, 0), (8, 5, 0), (8, 8, 0),
                                        (16, 32, 2), (16, 32, 0), (8, 64, 8), (6, 64, 2)])
def test_split_bit_exact_against_the_oracle(L, T, groups):
    n_runs, n_steps, seed = 3, 12, 0x5911 + T
    log(f"split PT L={L} T={T} groups={groups} runs={n_runs}")
    inst, Jo, go, egs = instance(L, seed + L, 0)
    thr, thrx = _ladder(T)
    out = sg.pt_run(inst, dev_u32(thr), dev_u32(thrx), n_runs, n_steps, seed, want_trace=True, want_swaps=True,
                    groups=groups)
    torch.cuda.synchronize()
    assert _status(out) == 0
    _check_oracle(L, Jo, _host(out), seed, range(n_runs), thr, thrx, n_steps)


@pytest.mark.parametrize("groups,waves", [(2, 0), (4, 0), (8, 0), (2, 8), (2, 16), (4, 4), (8, 12)])
def test_split_equals_pt_run_on_ragged_run_counts(groups, waves):
    L, T, n_runs, n_steps, seed = 8, 16, 13, 40, 0x77
    log(f"split PT vs pt_run L={L} T={T} runs={n_runs} groups={groups} waves={waves}")
    inst, Jo, go, egs = instance(L, 31, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    ref = sg.pt_run(inst, thr, thrx, n_runs, n_steps, seed, run0=5, want_trace=True, want_swaps=True)
    out = sg.pt_run(inst, thr, thrx, n_runs, n_steps, seed, run0=5, want_trace=True, want_swaps=True,
                    groups=groups, waves=waves)
    torch.cuda.synchronize()
    assert _status(out) == 0
    for k in ("spins", "energy", "pos", "emin_trace", "swap_acc"):
        assert torch.equal(out[k], ref[k]), k


def test_split_resume_equals_uninterrupted():
    L, T = 10, 8
    log("split PT resume")
    inst, Jo, go, egs = instance(L, 23, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    full = sg.pt_run(inst, thr, thrx, 4, 20, 7, run0=9, groups=4)
    a = sg.pt_run(inst, thr, thrx, 4, 8, 7, run0=9, groups=2)
    b = sg.pt_run(inst, thr, thrx, 4, 12, 7, run0=9, step0=8, spins=a["spins"].clone(), pos=a["pos"].clone(),
                  groups=8)
    torch.cuda.synchronize()
    assert _status(full) == 0 and _status(a) == 0 and _status(b) == 0
    for k in ("spins", "energy", "pos"):
        assert torch.equal(full[k], b[k]), k


@pytest.mark.parametrize("L,T,groups,waves", [(12, 32, 2, 0), (12, 32, 2, 8), (16, 16, 2, 12)])
def test_split_resume_with_drawn_colour0_words(L, T, groups, waves):
    # shapes whose lanes draw the next step's colour-0 words during the
    # trade (12 waves: up to two units per lane; 8 waves: three, as 1152
    # units over 512 lanes), resumed at a step other than 0: equal to one
    # uninterrupted one-group pt_run
    n_runs, seed = 3, 0x3141
    log(f"split PT resume with drawn words L={L} T={T} groups={groups} waves={waves}")
    inst, Jo, go, egs = instance(L, 17, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    ref = sg.pt_run(inst, thr, thrx, n_runs, 15, seed, run0=2)
    a = sg.pt_run(inst, thr, thrx, n_runs, 6, seed, run0=2, groups=groups, waves=waves)
    b = sg.pt_run(inst, thr, thrx, n_runs, 9, seed, run0=2, step0=6, spins=a["spins"].clone(),
                  pos=a["pos"].clone(), groups=groups, waves=waves)
    torch.cuda.synchronize()
    assert _status(a) == 0 and _status(b) == 0
    for k in ("spins", "energy", "pos"):
        assert torch.equal(b[k], ref[k]), k


def test_split_reuses_its_workspace():
    # the mailbox keeps the last call's tags; the next call clears it first
    L, T = 8, 8
    inst, Jo, go, egs = instance(L, 3, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    ws = torch.empty((sg.pt_split_workspace_bytes(16, T) + 7) // 8, dtype=torch.int64, device="cuda")
    ref = sg.pt_run(inst, thr, thrx, 16, 30, 99)
    for n_steps in (30, 12, 30):
        out = sg.pt_run(inst, thr, thrx, 16, n_steps, 99, groups=4, workspace=ws)
        torch.cuda.synchronize()
        assert _status(out) == 0
    for k in ("spins", "energy", "pos"):
        assert torch.equal(out[k], ref[k]), k


def test_split_pt_workload_full_size():
    # the PT workload (128 runs x 2000 steps, 32 temperatures, L = 12) with
    # the group count the bench uses: every run equals pt_run's, and run 77
    # is re-run by the oracle
    w = wl.pt()
    log("split PT workload full size", w.n_runs, w.n_steps)
    inst, Jo, go, egs = instance(w.instance.L, w.instance.seed, 0)
    thr, thrx = _ladder(w.T, (w.beta0, w.beta1))
    dthr, dthrx = dev_u32(thr), dev_u32(thrx)
    ref = sg.pt_run(inst, dthr, dthrx, w.n_runs, w.n_steps, w.seed, want_trace=True, want_swaps=True)
    out = sg.pt_run(inst, dthr, dthrx, w.n_runs, w.n_steps, w.seed, want_trace=True, want_swaps=True, groups=0)
    torch.cuda.synchronize()
    assert _status(out) == 0
    for k in ("spins", "energy", "pos", "emin_trace", "swap_acc"):
        assert torch.equal(out[k], ref[k]), k
    _check_oracle(w.instance.L, Jo, _host(out), w.seed, [77], thr, thrx, w.n_steps)


def test_ladder_beyond_one_groups_lds():
    # 32 walkers of L = 16 do not fit one work group's LDS: pt_run refuses,
    # the split form runs them (checked against the oracle above)
    L, T = 16, 32
    inst, Jo, go, egs = instance(L, 5, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    with pytest.raises(sg.SgError):
        sg.pt_run(inst, thr, thrx, 1, 2, 1)
    out = sg.pt_run(inst, thr, thrx, 1, 2, 1, groups=2)
    torch.cuda.synchronize()
    assert _status(out) == 0


def test_split_pt_captured_in_a_graph_replays_exactly():
    # the call (mailbox fill kernel + PT kernel) captured once; every replay,
    # with eager work on the device between replays, equals the eager call
    L, T, n_runs, n_steps = 8, 16, 13, 20
    log("split PT graph capture")
    inst, Jo, go, egs = instance(L, 41, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    ws = torch.empty((sg.pt_split_workspace_bytes(n_runs, T) + 7) // 8, dtype=torch.int64, device="cuda")
    ref = sg.pt_run(inst, thr, thrx, n_runs, n_steps, 42, want_trace=True, want_swaps=True, groups=4, workspace=ws)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items() if k != "workspace" and v is not None}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up on a side stream before the capture
        sg.pt_run(inst, thr, thrx, n_runs, n_steps, 42, groups=4, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        out = sg.pt_run(inst, thr, thrx, n_runs, n_steps, 42, want_trace=True, want_swaps=True, groups=4,
                        workspace=ws)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert _status(out) == 0, rep
        # (swap_acc is zeroed by a fill kernel captured with the call)
        for k in ("spins", "energy", "pos", "emin_trace", "swap_acc"):
            assert torch.equal(out[k], ref[k]), (rep, k)
        other = sg.pt_run(inst, thr, thrx, 3, 5, 7, groups=2, workspace=ws)   # eager, same workspace
        torch.cuda.synchronize()
        assert _status(other) == 0


def test_split_argument_errors():
    L, T = 8, 6
    inst, Jo, go, egs = instance(L, 1, 0)
    thr, thrx = (dev_u32(a) for a in _ladder(T))
    for groups, waves in ((3, 0), (4, 0), (2, 5)):
        with pytest.raises(sg.SgError):
            sg.pt_run(inst, thr, thrx, 2, 4, 1, groups=groups, waves=waves)
    small = torch.empty(4, dtype=torch.int64, device="cuda")
    with pytest.raises(sg.SgError):
        sg.pt_run(inst, thr, thrx, 2, 4, 1, groups=2, workspace=small)


@pytest.mark.parametrize("groups", [1, 2])
def test_pos_that_is_not_a_permutation_falls_back_to_identity(groups):
    # a caller's pos with a repeated slot (bypassing the binding's check,
    # straight through the C ABI): the run starts from the identity order
    # instead, so it equals a run given the identity, and the split form's
    # status word carries bit 1
    import ctypes
    L, T, n_runs, n_steps, seed = 8, 8, 2, 9, 0xB0B
    log(f"PT bad pos groups={groups}")
    inst, Jo, go, egs = instance(L, 0xB0B0 + groups, 0)
    thr, thrx = _ladder(T)
    dthr, dthrx = dev_u32(thr), dev_u32(thrx)
    start = sg.pt_run(inst, dthr, dthrx, n_runs, 3, seed)
    sp0 = start["spins"].clone()
    ident = torch.arange(T, dtype=torch.int32, device="cuda").repeat(n_runs, 1).contiguous()
    ref = sg.pt_run(inst, dthr, dthrx, n_runs, n_steps, seed, step0=3, spins=sp0.clone(), pos=ident.clone(),
                    want_trace=True, groups=groups)
    bad = ident.clone()
    bad[0, 3] = 5                         # slot 5 twice, slot 3 empty
    bad[1, 0] = T + 4                     # out of range
    sp = sp0.clone()
    en = torch.empty((n_runs, T), dtype=torch.int32, device="cuda")
    tr = torch.empty((n_runs, n_steps), dtype=torch.int32, device="cuda")
    args = sg.sg_pt_args(n_runs=n_runs, run0=0, T=T, n_steps=n_steps, step0=3, K=int(dthr.shape[1]),
                         M=int(dthrx.shape[1]), init_random=0, seed=seed)
    nb = sg.pt_split_workspace_bytes(n_runs, T)
    ws = torch.empty((nb + 7) // 8, dtype=torch.int64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = sg.lib().sg_pt_run_split(ctypes.byref(inst.struct()), ctypes.byref(args), groups, 0, p(dthr), p(dthrx),
                                  p(sp), p(en), p(bad), p(tr), None, p(ws), nb,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert int(ws.view(torch.int32)[0].item()) == 2
    assert torch.equal(sp, ref["spins"]) and torch.equal(en, ref["energy"])
    assert torch.equal(bad, ref["pos"]) and torch.equal(tr, ref["emin_trace"])
    with pytest.raises(sg.SgError):
        sg.pt_run(inst, dthr, dthrx, n_runs, 2, seed, spins=sp0.clone(), pos=ident.flip(1).contiguous() * 0)
