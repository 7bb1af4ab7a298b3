"""Batched annealing (sg_batch_*): a plan of mixed-L jobs, launched
directly or replayed as a hipGraph, gives every job exactly the result of
its own sa_anneal call; sampled replicas match the oracle."""
import numpy as np
import pytest
import torch

import paper_2501_17267_amd as sg
from paper_2501_17267_amd import workloads as wl
from gpu_util import dev_u32, log, oracle_sa_parallel

pytestmark = pytest.mark.gpu


def _jobs(n, seed):
    specs = wl.uneven(n_inst=n, n_rep=13, budgets=(5, 9, 16))
    insts, thr, host = [], {}, []
    for j in specs:
        J, g, egs = sg.make_instance(j.inst.L, 6, j.inst.seed)
        host.append(J)
        insts.append(sg.Instance(j.inst.L, J, egs, j.inst.chain))
        if j.n_sweeps not in thr:
            thr[j.n_sweeps] = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, j.n_sweeps))
    dthr = {S: dev_u32(t) for S, t in thr.items()}
    jobs = [sg.SAJob(inst, dthr[j.n_sweeps], j.n_rep, seed, rep0=3 * k, want_emin=(k % 3 == 0))
            for k, (inst, j) in enumerate(zip(insts, specs))]
    return specs, insts, host, thr, dthr, jobs


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_individual_calls(graph):
    log(f"batch vs plain graph={graph}")
    specs, insts, host, thr, dthr, jobs = _jobs(40, 0xBA7C)
    b = sg.Batch(jobs, graph=graph)
    for _ in range(2):   # replays give the same results
        b.launch()
        torch.cuda.synchronize()
        for k, (inst, j, job) in enumerate(zip(insts, specs, jobs)):
            sp, en, em = sg.sa_anneal(inst, dthr[j.n_sweeps], j.n_rep, 0xBA7C, rep0=3 * k,
                                      want_emin=job.emin is not None)
            torch.cuda.synchronize()
            assert torch.equal(sp, job.spins), k
            assert torch.equal(en, job.energy), k
            if job.emin is not None:
                assert torch.equal(em, job.emin), k
    info = b.info()
    assert info["kernels"] == len({j.inst.L for j in specs})
    b.close()


def test_batch_sampled_against_oracle():
    specs, insts, host, thr, dthr, jobs = _jobs(24, 0xFACE)
    b = sg.Batch(jobs, graph=True)
    b.launch()
    torch.cuda.synchronize()
    for k in (0, 5, 11, 23):
        j = specs[k]
        ref = oracle_sa_parallel(j.inst.L, host[k], 0xFACE, j.inst.chain, thr[j.n_sweeps],
                                 [3 * k, 3 * k + 12])
        sp, en = jobs[k].spins.cpu().numpy(), jobs[k].energy.cpu().numpy()
        for r in (0, 12):
            np.testing.assert_array_equal(sp[r], ref[3 * k + r][0])
            assert en[r] == ref[3 * k + r][1]
    b.close()
