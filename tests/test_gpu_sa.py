"""GPU parity of simulated annealing (sa_anneal through the C ABI) against
the oracle: bit-exact final spins, energies and best-seen energies."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from paper_2501_17267_amd import workloads as wl
from gpu_util import dev_u32, instance, log, oracle_sa_parallel

pytestmark = pytest.mark.gpu
K = 24


def _run_and_compare(L, n_rep, S, seed, chain=3, rep0=0, want_emin=True, sweep0=0, sample=None,
                     beta=(0.1, 3.0)):
    log(f"SA parity L={L} n_rep={n_rep} S={S} seed={seed:#x} rep0={rep0} emin={want_emin}")
    inst, Jo, go, egs = instance(L, seed * 7 + L, chain)
    thr = sg.make_thresholds(sg.make_schedule(0, beta[0], beta[1], S), K)
    sp, en, em = sg.sa_anneal(inst, dev_u32(thr), n_rep, seed, rep0=rep0, sweep0=sweep0,
                              want_emin=want_emin)
    torch.cuda.synchronize()
    sp, en = sp.cpu().numpy(), en.cpu().numpy()
    em = em.cpu().numpy() if em is not None else None
    reps = list(range(n_rep)) if sample is None else sample
    ref = oracle_sa_parallel(L, Jo, seed, chain, thr, [rep0 + r for r in reps], sweep0=sweep0,
                             want_emin=want_emin)
    for r in reps:
        s_ref, e_ref, m_ref = ref[rep0 + r]
        np.testing.assert_array_equal(sp[r], s_ref, err_msg=f"spins L={L} r={r}")
        assert en[r] == e_ref, (L, r)
        if want_emin:
            assert em[r] == m_ref, (L, r)
    assert np.all(en >= egs)
    return sp, en


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24])
def test_sa_bit_exact_every_lattice_size(L):
    # several groups plus a ragged last group, a few sweeps of the anneal
    n_rep = {4: 37, 6: 70, 8: 35, 10: 67, 12: 35, 14: 65, 16: 19, 18: 11, 20: 9, 22: 6, 24: 5}[L]
    _run_and_compare(L, n_rep, 6, 0xA11CE + L, want_emin=True)


@pytest.mark.parametrize("L", [26, 28, 30, 32, 64])
def test_sa_bit_exact_large_lattices(L):
    # couplings streamed from the encoded HBM buffer; spins in LDS up to
    # L = 32 and in the global workspace at L = 64
    n_rep = {26: 5, 28: 3, 30: 3, 32: 3, 64: 2}[L]
    _run_and_compare(L, n_rep, 3 if L == 64 else 4, 0xB16 + L, want_emin=True)


@pytest.mark.parametrize("L", [34, 40, 50, 56, 62])
def test_sa_bit_exact_paper_scaling_sizes(L):
    # the sizes of the paper's annealing scaling study (App. D: L = 20 ... 56)
    # and the ones between 32 and 64: spins in the workspace, couplings from
    # the encoded image, one replica per work group; L = 34, 50, 62 have the
    # half-used last column dword (L = 2 mod 4)
    _run_and_compare(L, 2, 3, 0xC0DE + L, want_emin=True)


@pytest.mark.parametrize("L", [26, 28, 30, 32, 34, 40, 50, 56, 64])
def test_sa_wide_path_bit_exact(L):
    # few replicas without the best-seen energy: sa_anneal spreads each
    # colour phase over the device (one lane per column dword)
    n_rep = {26: 3, 28: 2, 30: 3, 32: 2, 34: 3, 40: 2, 50: 3, 56: 2, 64: 2}[L]
    assert sg.sa_wide_workspace_bytes(L, n_rep) > 0
    _run_and_compare(L, n_rep, 3 if L == 64 else 5, 0xD1DE + L, want_emin=False)


@pytest.mark.parametrize("L", [30, 50, 64])
def test_sa_wide_explicit_offsets_resume_and_equality_with_group_kernel(L):
    # explicit wide entry point: replica and sweep offsets, a start from
    # given spins, and equality with the single-work-group kernel
    inst, Jo, go, egs = instance(L, 0x5EED + L, 4)
    S = 4 if L == 64 else 6
    thr = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 2 * S), K)
    log(f"SA wide explicit L={L}")
    n_rep = 5
    a_s, a_e = sg.sa_anneal_wide(inst, dev_u32(thr[:S]), n_rep, 0x77, rep0=9)
    b_s, b_e = sg.sa_anneal_wide(inst, dev_u32(thr[S:]), n_rep, 0x77, rep0=9, sweep0=S, spins=a_s.clone())
    g_s, g_e, _ = sg.sa_anneal_variant(inst, dev_u32(thr), n_rep, 0x77, 0, rep0=9)
    torch.cuda.synchronize()
    assert torch.equal(b_s, g_s) and torch.equal(b_e, g_e)
    ref = oracle_sa_parallel(L, Jo, 0x77, 4, thr, [9, 13])
    sp, en = b_s.cpu().numpy(), b_e.cpu().numpy()
    for r, rr in ((0, 9), (4, 13)):
        np.testing.assert_array_equal(sp[r], ref[rr][0])
        assert en[r] == ref[rr][1]


@pytest.mark.parametrize("L", [8, 12])
def test_sa_bit_exact_without_tracking_and_with_offsets(L):
    _run_and_compare(L, 20, 9, 0xBEE + L, rep0=1000, sweep0=77, want_emin=False)


def test_sa_small_workload_full():
    # the L=4 workload: 64 restarts x 1000 sweeps, every replica bit-exact
    w = wl.sa_small()
    spec = w.instances[0]
    inst, Jo, go, egs = instance(spec.L, spec.seed, spec.chain)
    thr = sg.make_thresholds(sg.make_schedule(0, w.beta0, w.beta1, w.n_sweeps), K)
    log("sa_small full", spec.L, w.n_rep, w.n_sweeps)
    sp, en, em = sg.sa_anneal(inst, dev_u32(thr), w.n_rep, w.seed, want_emin=True)
    torch.cuda.synchronize()
    ref = oracle_sa_parallel(spec.L, Jo, w.seed, spec.chain, thr, list(range(w.n_rep)), want_emin=True)
    sp, en, em = sp.cpu().numpy(), en.cpu().numpy(), em.cpu().numpy()
    for r in range(w.n_rep):
        np.testing.assert_array_equal(sp[r], ref[r][0])
        assert en[r] == ref[r][1] and em[r] == ref[r][2]
    eps = sg.epsilon(torch.from_numpy(en).cuda(), egs).cpu().numpy()
    assert np.all(eps >= 0)


@pytest.mark.parametrize("L", [8, 12, 16])
def test_sa_batch_sizes_full_replica_count_sampled(L):
    # one instance of the batched workload at full size (1024 replicas x 256
    # sweeps); every replica is an independent chain, so sampled replicas
    # are compared one by one (first, last, a middle block)
    w = wl.sa_batch()
    spec = [s for s in w.instances if s.L == L][0]
    inst, Jo, go, egs = instance(L, spec.seed, spec.chain)
    thr = sg.make_thresholds(sg.make_schedule(0, w.beta0, w.beta1, w.n_sweeps), K)
    log("sa_batch instance full size", L, w.n_rep, w.n_sweeps)
    sp, en, _ = sg.sa_anneal(inst, dev_u32(thr), w.n_rep, w.seed)
    torch.cuda.synchronize()
    sp, en = sp.cpu().numpy(), en.cpu().numpy()
    reps = [0, 1, 511, 512, 1023]
    ref = oracle_sa_parallel(L, Jo, w.seed, spec.chain, thr, reps)
    for r in reps:
        np.testing.assert_array_equal(sp[r], ref[r][0])
        assert en[r] == ref[r][1]
    # energies of all replicas agree with an independent recomputation
    en2 = sg.energy(inst, torch.from_numpy(sp).cuda()).cpu().numpy()
    np.testing.assert_array_equal(en, en2)


def test_sa_chunked_equals_monolithic_and_resume_from_spins():
    L = 12
    inst, Jo, go, egs = instance(L, 99, 5)
    thr = sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 40), K)
    full_s, full_e, _ = sg.sa_anneal(inst, dev_u32(thr), 33, 1234)
    a_s, a_e, _ = sg.sa_anneal(inst, dev_u32(thr[:15]), 33, 1234)
    b_s, b_e, _ = sg.sa_anneal(inst, dev_u32(thr[15:]), 33, 1234, sweep0=15, spins=a_s.clone())
    torch.cuda.synchronize()
    assert torch.equal(full_s, b_s) and torch.equal(full_e, b_e)


def test_sa_planted_start_at_zero_temperature_stays_planted():
    # the planted state is a ground state: at beta = infinity nothing moves
    # uphill and eps stays exactly 0
    L = 16
    inst, Jo, go, egs = instance(L, 4242, 1)
    thr = np.zeros((5, K), np.uint32)
    start = torch.from_numpy(np.tile(go, (3, 1))).cuda()
    sp, en, _ = sg.sa_anneal(inst, dev_u32(thr), 3, 77, spins=start.clone())
    eps = sg.epsilon(en, egs)
    torch.cuda.synchronize()
    assert np.all(en.cpu().numpy() == egs)
    assert np.all(eps.cpu().numpy() == 0.0)


def test_sa_encoded_couplings_path_matches_plain():
    L = 10
    inst, Jo, go, egs = instance(L, 555, 2)
    inst_enc = sg.Instance(L, inst.J, egs, 2, encode=True)
    thr = dev_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 12), K))
    a = sg.sa_anneal(inst, thr, 40, 9)
    b = sg.sa_anneal(inst_enc, thr, 40, 9)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
