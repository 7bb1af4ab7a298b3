"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, its host helpers (schedules, acceptance tables, the
tile-planted generator) agree bit for bit with the oracle, and invalid
arguments are refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2501_17267_amd as sg


def test_library_exports_every_header_function():
    lib = sg.lib()
    names = sg.header_functions()
    assert {"sa_anneal", "pt_run", "energy", "epsilon"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_and_version():
    lib = sg.lib()
    assert lib.sg_strerror(0) == b"ok"
    assert lib.sg_strerror(-1) == b"invalid argument"
    assert b"gfx950" in lib.sg_version()


@pytest.mark.parametrize("kind,b0,b1,S", [(0, 0.1, 3.0, 1000), (0, 0.1, 3.0, 256), (1, 0.2, 3.0, 32),
                                          (1, 0.3, 27.0, 977), (0, 5.0, 5.0, 3), (0, 0.7, 9.0, 1)])
def test_schedule_and_thresholds_match_oracle(kind, b0, b1, S):
    beta = sg.make_schedule(kind, b0, b1, S)
    np.testing.assert_array_equal(beta, oracle.schedule(kind, b0, b1, S))
    for K in (1, 6, 24):
        np.testing.assert_array_equal(sg.make_thresholds(beta, K), oracle.thresholds(beta, K))


def test_exchange_tables_match_oracle():
    beta = sg.make_schedule(1, 0.2, 3.0, 32)
    M = sg.exchange_table_width(beta)
    assert M == 607
    np.testing.assert_array_equal(sg.make_exchange_thresholds(beta, M), oracle.exchange_thresholds(beta, M))
    ref = oracle.exchange_thresholds(beta, M + 50)
    assert np.all(ref[:, M:] == 0)
    assert np.any(ref[:, M - 1] != 0)


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14, 16, 20, 24, 32])
@pytest.mark.parametrize("cls", [6, 2, -1])
def test_instance_generator_matches_oracle(L, cls):
    seed = 0x9E37 * L + cls + 1000
    J, g, egs = sg.make_instance(L, cls, seed)
    Jo, go, egso = oracle.make_instance(L, cls, seed)
    np.testing.assert_array_equal(J, Jo)
    np.testing.assert_array_equal(g, go)
    assert egs == egso


def test_instance_generator_large_lattice_matches_oracle():
    J, g, egs = sg.make_instance(64, 6, 12345)
    Jo, go, egso = oracle.make_instance(64, 6, 12345)
    np.testing.assert_array_equal(J, Jo)
    assert egs == egso
    assert oracle.energy(Jo, go, (64, 64, 64)) == egs


def test_wide_workspace_size():
    # spins of n_rep replicas in the column layout, where the automatic
    # choice takes the multi-work-group path: the selected single-group
    # kernel would launch fewer than 128 replica groups
    for L in (26, 28, 30, 32, 34, 40, 50, 56, 62, 64):
        C = (L + 3) // 4
        rpw = sg.sa_variants(L)[sg.selected_variant(L)]["replicas_per_group"]
        for n in (1, 3, 16, 127 * rpw, 127 * rpw + 1, 128 * rpw):
            want = n * L * L * C * 4 if -(-n // rpw) < 128 else 0
            assert sg.sa_wide_workspace_bytes(L, n) == want, (L, n)
    assert sg.sa_wide_workspace_bytes(24, 1) == 0
    assert sg.sa_wide_workspace_bytes(40, 1) == 40 * 40 * 10 * 4
    assert sg.sa_wide_workspace_bytes(66, 1) == 0
    assert sg.sa_wide_workspace_bytes(32, 0) == 0


def test_jenc_size():
    for L in (4, 6, 12, 16, 64):
        H, C = L // 2, (L + 3) // 4
        assert sg.jenc_bytes(L) == 2 * (H * L) * 6 * 2 * C * 4
    assert sg.jenc_bytes(5) == 0


def _bad_call(fn, *args):
    rc = fn(*args)
    return rc, sg.lib().sg_last_error().decode()


def test_invalid_arguments_are_refused_on_the_host():
    lib = sg.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    inst = sg.sg_instance(L=5, J=0x1000, E_gs=-10)
    args = sg.sg_sa_args(n_rep=4, n_sweeps=8, K=24, init_random=1, seed=1)
    rc, msg = _bad_call(lib.sa_anneal, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None)
    assert rc == -1 and "L = 5" in msg
    inst.L = 8
    args.K = 25
    assert lib.sa_anneal(ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None) == -1
    args.K = 24
    args.n_rep = 0
    assert lib.sa_anneal(ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None) == -1
    args.n_rep = 4
    args.sweep0 = (1 << 30)
    assert lib.sa_anneal(ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None) == -4
    args.sweep0 = 0
    assert lib.sa_anneal(ctypes.byref(inst), ctypes.byref(args), fake, ctypes.c_void_p(0x1001), fake,
                         None, None) == -1
    assert lib.sa_anneal(None, ctypes.byref(args), fake, fake, fake, None, None) == -1
    inst.L = 32   # supported, but only with the encoded couplings
    rc, msg = _bad_call(lib.sa_anneal, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None)
    assert rc == -1 and "encoded couplings" in msg
    inst.L = 64   # also needs a workspace
    inst.jenc = 0x2000
    rc, msg = _bad_call(lib.sa_anneal, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None)
    assert rc == -1 and "workspace" in msg
    assert lib.sg_sa_workspace_bytes(64, 3) == 3 * 2 * 2048 * 16 * 4
    assert lib.sg_sa_workspace_bytes(32, 3) == 0
    inst.L = 40   # every even size up to 64 has a kernel; above 32 it needs a workspace
    rc, msg = _bad_call(lib.sa_anneal, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None)
    assert rc == -1 and "workspace" in msg
    assert lib.sg_sa_workspace_bytes(50, 2) == 2 * 2 * (25 * 50) * 13 * 4
    for L in range(34, 64, 2):
        assert lib.sg_sa_variants(L, 0, None) >= 1, L
    inst.L = 66   # beyond SG_MAX_L
    rc, msg = _bad_call(lib.sa_anneal, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None, None)
    assert rc == -1 and "L = 66" in msg
    # the multi-work-group path: even L = 26..64 only, with a large enough
    # 16-byte aligned workspace
    inst.L = 16
    rc, msg = _bad_call(lib.sg_sa_anneal_wide, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None)
    assert rc == -7 and "wide" in msg
    inst.L = 32
    rc, msg = _bad_call(lib.sg_sa_anneal_wide, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None)
    assert rc == -1 and "workspace" in msg
    args.workspace = 0x3000
    args.workspace_bytes = 4 * 32 * 32 * 8 * 4 - 4
    assert lib.sg_sa_anneal_wide(ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None) == -1
    args.workspace_bytes += 4
    args.workspace = 0x3004
    rc, msg = _bad_call(lib.sg_sa_anneal_wide, ctypes.byref(inst), ctypes.byref(args), fake, fake, fake, None)
    assert rc == -1 and "aligned" in msg
    args.workspace, args.workspace_bytes = None, 0
    inst.jenc = None
    # fragment decimation: shape rules checked before any launch
    inst.L = 12
    inst.J = 0x1000
    fa = sg.sg_frag_args(core=1, halo=2, replicas=4, order=1, n_runs=2, n_sweeps=10, K=24, seed=1)
    for field, bad in (("core", 5), ("halo", 6), ("replicas", 17), ("replicas", 0), ("order", 2),
                       ("n_runs", 0), ("K", 25)):
        old = getattr(fa, field)
        setattr(fa, field, bad)
        rc, msg = _bad_call(lib.sg_fragment_decimate, ctypes.byref(inst), ctypes.byref(fa), fake, fake, None, None)
        assert rc == -1, (field, bad, rc, msg)
        setattr(fa, field, old)
    fa.core, fa.halo, fa.order = 4, 1, 0   # 3 cores per axis cannot be 2-coloured
    rc, msg = _bad_call(lib.sg_fragment_decimate, ctypes.byref(inst), ctypes.byref(fa), fake, fake, None, None)
    assert rc == -1 and "divisible" in msg
    fa.core, fa.halo, fa.order = 1, 4, 1   # l = 9 is allowed at L = 12, l = 11 is not
    fa.halo = 5
    assert lib.sg_fragment_decimate(ctypes.byref(inst), ctypes.byref(fa), fake, fake, None, None) == -1
    fa.halo, fa.run0 = 2, 0xFFFFFFFF
    assert lib.sg_fragment_decimate(ctypes.byref(inst), ctypes.byref(fa), fake, fake, None, None) == -4
    inst.J = None
    fa.run0 = 0
    assert lib.sg_fragment_decimate(ctypes.byref(inst), ctypes.byref(fa), fake, fake, None, None) == -1
    # PT
    inst.L = 12
    pargs = sg.sg_pt_args(n_runs=2, T=1, n_steps=5, K=24, M=10, init_random=1, seed=3)
    assert lib.pt_run(ctypes.byref(inst), ctypes.byref(pargs), fake, fake, fake, fake, fake, None, None,
                      None) == -1
    pargs.T = 65
    assert lib.pt_run(ctypes.byref(inst), ctypes.byref(pargs), fake, fake, fake, fake, fake, None, None,
                      None) == -1
    pargs.T = 8
    pargs.M = 0
    assert lib.pt_run(ctypes.byref(inst), ctypes.byref(pargs), fake, fake, fake, fake, fake, None, None,
                      None) == -1
    # energy / epsilon
    assert lib.energy(ctypes.byref(inst), 0, fake, fake, None) == -1
    assert lib.epsilon(fake, 10, 0, fake, None) == -1
    assert lib.epsilon(fake, 0, -5, fake, None) == -1
    # host helpers
    out = np.zeros(4, np.float64)
    assert lib.sg_make_schedule(1, 0.0, 3.0, 4, out.ctypes.data) == -1
    assert lib.sg_make_schedule(0, 0.1, 3.0, 0, out.ctypes.data) == -1
    thr = np.zeros(100, np.uint32)
    assert lib.sg_make_thresholds(out.ctypes.data, 4, 25, thr.ctypes.data) == -1
    assert lib.sg_make_instance(6, 3, 1, thr.ctypes.data, thr.ctypes.data, thr.ctypes.data) == -1


def test_split_pt_arguments_are_refused_on_the_host():
    lib = sg.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.sg_pt_split_workspace_bytes(128, 32) == 256 + 128 * 2 * 32 * 8
    assert lib.sg_pt_split_workspace_bytes(0, 32) == 0 and lib.sg_pt_split_workspace_bytes(4, 65) == 0
    inst = sg.sg_instance(L=12, J=0x1000, E_gs=-10)
    args = sg.sg_pt_args(n_runs=4, T=6, n_steps=10, K=24, M=8, init_random=1, seed=1)
    need = lib.sg_pt_split_workspace_bytes(4, 6)

    def call(groups, waves, ws, nbytes):
        return _bad_call(lib.sg_pt_run_split, ctypes.byref(inst), ctypes.byref(args), groups, waves, fake, fake,
                         fake, fake, fake, None, None, ws, nbytes, None)
    for groups, waves, ws, nbytes, text in ((3, 0, fake, need, "groups = 3"),
                                           (4, 0, fake, need, "multiple"),
                                           (2, 5, fake, need, "waves = 5"),
                                           (2, 0, None, 0, "workspace"),
                                           (2, 0, fake, need - 8, "needed"),
                                           (2, 0, ctypes.c_void_p(0x1004), need, "aligned")):
        rc, msg = call(groups, waves, ws, nbytes)
        assert rc == -1 and text in msg, (groups, waves, msg)
    args.T = 1
    rc, msg = call(2, 0, fake, need)
    assert rc == -1 and "T = 1" in msg


def test_static_split_pt_rejects_runs_beyond_its_array():
    # the no-allocation split PT refuses, before touching the device, a
    # mailbox larger than its fixed array (SG_ERANGE), and bad shapes
    lib = sg.lib()
    assert lib.sg_pt_split_workspace_bytes(1024, 64) > (1 << 20)
    args = sg.sg_pt_args(n_runs=1024, run0=0, T=64, n_steps=1, step0=0, K=24, M=1, init_random=1, seed=1)
    inst = sg.sg_instance(L=8, J=0x1000, jenc=None, E_gs=-10, chain=0)
    fake = ctypes.c_void_p(0x1000)
    rc, msg = _bad_call(lib.sg_pt_run_split_static, ctypes.byref(inst), ctypes.byref(args), 0, 0, fake, fake, fake,
                        fake, fake, None, None, None, None)
    assert rc == -4 and "static" in msg
    args.n_runs, args.T = 0, 8
    assert lib.sg_pt_run_split_static(ctypes.byref(inst), ctypes.byref(args), 0, 0, fake, fake, fake, fake, fake,
                                      None, None, None, None) == -1
