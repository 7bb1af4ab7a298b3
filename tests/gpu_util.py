"""Helpers of the GPU parity tests: device tables, instances and a thread
pool that runs independent oracle chains side by side on the host cores."""
import concurrent.futures as cf
import os
import sys

import numpy as np

import oracle
import paper_2501_17267_amd as sg

CORES = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))


def log(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev_u32(a):
    return sg.to_device_u32(a)


def instance(L, seed, chain=0, cls=6, encode=None):
    """Library-generated instance on the GPU plus the oracle's copy of J
    (encoded couplings are built automatically for L > 24)."""
    J, g, egs = sg.make_instance(L, cls, seed)
    Jo, go, egso = oracle.make_instance(L, cls, seed)
    assert np.array_equal(J, Jo) and egs == egso
    inst = sg.Instance(L, J, egs, chain, encode=encode)
    return inst, Jo, go, egs


def oracle_sa_parallel(L, J, seed, chain, thr, reps, sweep0=0, spins=None, want_emin=False):
    """Oracle chains for the replica counter words in `reps` (one call per
    replica, run on CORES threads).  spins: dict rep -> initial spins."""
    def one(r):
        s0 = None if spins is None else spins[r][None, :]
        sp, en, em = oracle.sa_run(L, J, seed, chain, thr, n_rep=1, rep0=r, sweep0=sweep0, spins=s0,
                                   want_emin=want_emin)
        return r, sp[0], int(en[0]), (int(em[0]) if em is not None else None)
    with cf.ThreadPoolExecutor(CORES) as ex:
        return {r: (s, e, m) for r, s, e, m in ex.map(one, reps)}
