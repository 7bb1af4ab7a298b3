"""GPU parity of the energy (Eq. 1) and optimality-gap (Eq. 2) kernels and
of the instance checks."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from gpu_util import instance, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [4, 6, 12, 32, 64])
def test_energy_kernel_matches_oracle(L):
    log("energy parity", L)
    inst, Jo, go, egs = instance(L, 31 + L, 0)
    rng = np.random.default_rng(L)
    n = 5 if L < 64 else 2
    s = rng.choice(np.array([-1, 1], np.int8), size=(n, L ** 3))
    s[0] = go
    e = sg.energy(inst, torch.from_numpy(s).cuda()).cpu().numpy()
    for r in range(n):
        assert e[r] == oracle.energy(Jo, s[r], (L, L, L))
    assert e[0] == egs


def test_epsilon_kernel_bit_exact():
    rng = np.random.default_rng(3)
    E = rng.integers(-300000, 300000, size=5000).astype(np.int32)
    for egs in (-360, -123457, -3000001, 777):
        eps = sg.epsilon(torch.from_numpy(E).cuda(), egs).cpu().numpy()
        ref = np.array([oracle.epsilon(int(e), egs) for e in E])
        np.testing.assert_array_equal(eps, ref)


def test_check_instance_flags_bad_couplings():
    L = 8
    inst, Jo, go, egs = instance(L, 8, 0)
    assert sg.check_instance(inst) == 0
    J = Jo.copy()
    J[0, 5] = 5              # out of range and breaks the pair copy
    bad = sg.Instance(L, J, egs, 0)
    assert sg.check_instance(bad) > 0
    J = Jo.copy()
    J[3, 17] = -J[3, 17] if J[3, 17] != 0 else 1   # only the pair copy broken
    bad = sg.Instance(L, J, egs, 0)
    assert sg.check_instance(bad) > 0


@pytest.mark.parametrize("G,n,n_bins", [(1, 1, 1), (3, 257, 16), (40, 20, 64), (17, 1024, 1024), (2, 5000, 7)])
def test_epsilon_stats_bit_exact(G, n, n_bins):
    # per-group gap statistics (Eq. 2; App. D's TT-eps criterion) against the
    # oracle on the same energies: exact sums and extremes, target counts and
    # histograms decided in double on both sides
    log("epsilon_stats parity", G, n, n_bins)
    rng = np.random.default_rng(G * 1000 + n)
    egs = -rng.integers(1000, 400000, size=G).astype(np.int64)
    span = (np.abs(egs) * 0.3).astype(np.int64)
    # gaps from slightly below 0 (E < E_gs) to 0.3, past eps_max = 0.25
    E = (egs[:, None] + (rng.random((G, n)) * span[:, None]).astype(np.int64) - 3).astype(np.int32)
    E[:, 0] = egs                       # one trial at the ground state
    targets = (0.0, 0.01, 0.03, 0.05, 0.1, 0.2, 0.25, 0.3)
    st = sg.epsilon_stats(torch.from_numpy(E).cuda(), egs, targets=targets, eps_max=0.25, n_bins=n_bins)
    ref = oracle.eps_stats(E, egs, targets=targets, eps_max=0.25, n_bins=n_bins)
    np.testing.assert_array_equal(st["sum"].cpu().numpy(), ref["sum"])
    np.testing.assert_array_equal(st["emin"].cpu().numpy(), ref["emin"])
    np.testing.assert_array_equal(st["emax"].cpu().numpy(), ref["emax"])
    np.testing.assert_array_equal(st["n_le"].cpu().numpy(), ref["n_le"])
    np.testing.assert_array_equal(st["hist"].cpu().numpy().view(np.uint32), ref["hist"])
    m = sg.mean_epsilon(st, egs)
    ref_m = (ref["sum"] - n * egs).astype(np.float64) / (n * np.abs(egs).astype(np.float64))
    np.testing.assert_array_equal(m, ref_m)


def test_epsilon_stats_on_anneal_output_and_without_histogram():
    # the statistics of a real batched anneal, one group per instance
    log("epsilon_stats on anneal output")
    L, n_rep, S = 8, 96, 40
    thr_h = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S))
    thr = sg.to_device_u32(thr_h)
    insts = [instance(L, 900 + k, k) for k in range(5)]
    E = torch.empty((5, n_rep), dtype=torch.int32, device="cuda")
    for k, (inst, Jo, go, egs) in enumerate(insts):
        sp, en, _ = sg.sa_anneal(inst, thr, n_rep, 0xE95)
        E[k] = en
    egs = [x[3] for x in insts]
    st = sg.epsilon_stats(E, egs, targets=(0.02, 0.05))
    assert "hist" not in st
    ref = oracle.eps_stats(E.cpu().numpy(), egs, targets=(0.02, 0.05))
    np.testing.assert_array_equal(st["sum"].cpu().numpy(), ref["sum"])
    np.testing.assert_array_equal(st["n_le"].cpu().numpy(), ref["n_le"])
    # a replica of the oracle's chain for instance 0 pins the energies too
    Jo = insts[0][1]
    _, e_or, _ = oracle.sa_run(L, Jo, 0xE95, 0, thr_h, n_rep=3)
    np.testing.assert_array_equal(E[0, :3].cpu().numpy().astype(np.int64), e_or)


def test_epsilon_stats_rejects_bad_arguments():
    E = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(sg.SgError):
        sg.epsilon_stats(E, [-5, -5], targets=tuple(range(9)))
    with pytest.raises(sg.SgError):
        sg.epsilon_stats(E, [-5, -5], eps_max=0.0, n_bins=4)
    with pytest.raises(sg.SgError):
        sg.epsilon_stats(E, [-5, -5], eps_max=1.0, n_bins=2000)
