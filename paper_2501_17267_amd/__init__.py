"""paper_2501_17267_amd -- Python binding of libsgmi (MI355X annealing of
cubic-lattice Ising spin glasses).

Argument marshalling only: every step of the annealing path runs in the HIP
kernels of ``libsgmi.so`` behind the C ABI declared in ``include/sgmi.h``.
PyTorch supplies device memory and the current stream.  The library must be
built (``python -m paper_2501_17267_amd.build``); importing the binding
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgmi.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "sgmi.h")

SG_OK = 0
SG_EINVAL = -1
SG_EBUSY = -5
SG_MAX_L = 64
SG_K_MAX = 24
SG_LDS_MAX_L = 24
SG_PT_MAX_T = 64


class SgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class sg_instance(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("J", ctypes.c_void_p), ("jenc", ctypes.c_void_p),
                ("E_gs", ctypes.c_int64), ("chain", ctypes.c_uint32),
                ("reserved2", ctypes.c_uint32)]


class sg_sa_args(ctypes.Structure):
    _fields_ = [("n_rep", ctypes.c_int32), ("rep0", ctypes.c_uint32),
                ("n_sweeps", ctypes.c_int32), ("sweep0", ctypes.c_int32),
                ("K", ctypes.c_int32), ("init_random", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_int64)]


class sg_sa_job(ctypes.Structure):
    _fields_ = [("inst", sg_instance), ("args", sg_sa_args), ("thr", ctypes.c_void_p),
                ("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p), ("emin", ctypes.c_void_p)]


class sg_pticm_args(ctypes.Structure):
    _fields_ = [("n_runs", ctypes.c_int32), ("run0", ctypes.c_uint32), ("T", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("step0", ctypes.c_int32), ("K", ctypes.c_int32),
                ("M", ctypes.c_int32), ("init_random", ctypes.c_int32), ("icm_from", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class sg_frag_args(ctypes.Structure):
    _fields_ = [("core", ctypes.c_int32), ("halo", ctypes.c_int32), ("replicas", ctypes.c_int32),
                ("order", ctypes.c_int32), ("n_runs", ctypes.c_int32), ("run0", ctypes.c_uint32),
                ("n_sweeps", ctypes.c_int32), ("K", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class sg_tn_plan_info(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("halo", ctypes.c_int32), ("order", ctypes.c_int32),
                ("lds_max_bits", ctypes.c_int32), ("n_phases", ctypes.c_int32), ("n_shapes", ctypes.c_int32),
                ("max_bits", ctypes.c_int32), ("n_lds_sites", ctypes.c_int32), ("n_hbm_sites", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("pair_updates", ctypes.c_double)]


class sg_tn_args(ctypes.Structure):
    _fields_ = [("J", ctypes.c_void_p), ("n_inst", ctypes.c_int32), ("tropical", ctypes.c_int32),
                ("beta", ctypes.c_double), ("spins_out", ctypes.c_void_p), ("score_out", ctypes.c_void_p),
                ("energy_out", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_int64)]


class sg_sa_variant(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("replicas_per_group", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("both_encodings", ctypes.c_int32),
                ("couplings_in_hbm", ctypes.c_int32), ("spins_in_hbm", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lds_bytes", ctypes.c_int64)]


class sg_sa_tune_result(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("identical", ctypes.c_int32), ("ms", ctypes.c_float),
                ("attempts_per_s", ctypes.c_double)]


SG_EPS_MAX_TARGETS = 8
SG_EPS_MAX_BINS = 1024


class sg_eps_stats(ctypes.Structure):
    _fields_ = [("energy_sum", ctypes.c_int64), ("energy_min", ctypes.c_int32), ("energy_max", ctypes.c_int32),
                ("n", ctypes.c_int32), ("n_le", ctypes.c_int32 * SG_EPS_MAX_TARGETS), ("reserved", ctypes.c_int32)]


class sg_pt_args(ctypes.Structure):
    _fields_ = [("n_runs", ctypes.c_int32), ("run0", ctypes.c_uint32),
                ("T", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("step0", ctypes.c_int32), ("K", ctypes.c_int32),
                ("M", ctypes.c_int32), ("init_random", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_lib = None


def header_functions() -> list[str]:
    """Names of every function the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return [n for n in names if n not in ("defined",)]


def lib() -> ctypes.CDLL:
    """Load libsgmi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2501_17267_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp = c.c_void_p
    L.sg_strerror.restype = c.c_char_p
    L.sg_strerror.argtypes = [c.c_int]
    L.sg_last_error.restype = c.c_char_p
    L.sg_last_error.argtypes = []
    L.sg_version.restype = c.c_char_p
    L.sg_make_schedule.argtypes = [c.c_int32, c.c_double, c.c_double, c.c_int32, vp]
    L.sg_make_thresholds.argtypes = [vp, c.c_int32, c.c_int32, vp]
    L.sg_make_exchange_thresholds.argtypes = [vp, c.c_int32, c.c_int32, vp]
    L.sg_exchange_table_width.argtypes = [vp, c.c_int32]
    L.sg_exchange_table_width.restype = c.c_int32
    L.sg_make_instance.argtypes = [c.c_int32, c.c_int32, c.c_uint64, vp, vp, vp]
    L.sg_sa_workspace_bytes.restype = c.c_size_t
    L.sg_sa_workspace_bytes.argtypes = [c.c_int32, c.c_int32]
    L.sg_sa_wide_workspace_bytes.restype = c.c_size_t
    L.sg_sa_wide_workspace_bytes.argtypes = [c.c_int32, c.c_int32]
    L.sg_sa_anneal_wide.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_sa_args), vp, vp, vp, vp]
    L.sg_jenc_bytes.restype = c.c_size_t
    L.sg_jenc_bytes.argtypes = [c.c_int32]
    L.sg_encode_instance.argtypes = [c.POINTER(sg_instance), vp, vp]
    L.sg_check_instance.argtypes = [c.POINTER(sg_instance), vp, vp]
    L.sa_anneal.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_sa_args), vp, vp, vp, vp, vp]
    L.pt_run.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_pt_args), vp, vp, vp, vp, vp, vp, vp, vp]
    L.sg_pt_run_split.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_pt_args), c.c_int32, c.c_int32, vp, vp, vp,
                                  vp, vp, vp, vp, vp, c.c_int64, vp]
    L.sg_pt_split_workspace_bytes.restype = c.c_size_t
    L.sg_pt_split_workspace_bytes.argtypes = [c.c_int32, c.c_int32]
    L.sg_pt_run_split_static.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_pt_args), c.c_int32, c.c_int32,
                                         vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.energy.argtypes = [c.POINTER(sg_instance), c.c_int32, vp, vp, vp]
    L.sg_pticm_run.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_pticm_args), vp, vp, vp, vp, vp, vp, vp,
                               vp, vp]
    L.sg_fragment_decimate.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_frag_args), vp, vp, vp, vp]
    L.sg_tn_plan_create.argtypes = [c.c_int32, c.c_int32, c.c_int32, c.c_int32, c.POINTER(c.c_void_p)]
    L.sg_tn_plan_info_get.argtypes = [vp, c.POINTER(sg_tn_plan_info)]
    L.sg_tn_plan_destroy.argtypes = [vp]
    L.sg_tn_plan_program.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.sg_tn_plan_rounds.argtypes = [vp, vp, vp, vp]
    L.sg_tn_workspace_bytes.argtypes = [vp, c.c_int32, c.c_int32]
    L.sg_tn_workspace_bytes.restype = c.c_int64
    L.sg_tn_decimate.argtypes = [vp, c.POINTER(sg_tn_args), vp]
    L.epsilon.argtypes = [vp, c.c_int64, c.c_int64, vp, vp]
    L.epsilon_stats.argtypes = [vp, c.c_int32, c.c_int32, vp, vp, c.c_int32, c.c_double, c.c_int32, vp, vp, vp]
    L.sg_batch_create.argtypes = [vp, c.c_int32, c.c_int32, c.POINTER(c.c_void_p)]
    L.sg_batch_launch.argtypes = [vp, vp]
    L.sg_batch_info.argtypes = [vp, vp, vp, vp]
    L.sg_batch_kernels.argtypes = [vp, c.c_int32, vp, vp, vp]
    L.sg_batch_destroy.argtypes = [vp]
    L.sg_sa_variants.argtypes = [c.c_int32, c.c_int32, vp]
    L.sg_sa_select_variant.argtypes = [c.c_int32, c.c_int32]
    L.sg_sa_selected_variant.argtypes = [c.c_int32]
    L.sg_sa_anneal_variant.argtypes = [c.POINTER(sg_instance), c.POINTER(sg_sa_args), vp, vp, vp, vp,
                                       c.c_int32, vp]
    L.sg_autotune_sa.argtypes = [c.c_int32, c.c_int32, c.c_int32, c.c_int32, vp, c.c_int32, vp]
    for fn in ("sg_sa_variants", "sg_sa_select_variant", "sg_sa_selected_variant",
               "sg_sa_anneal_variant", "sg_autotune_sa", "sg_batch_create", "sg_batch_launch", "sg_batch_info", "sg_batch_kernels",
               "sg_batch_destroy", "sg_make_schedule", "sg_make_thresholds", "sg_make_exchange_thresholds",
               "sg_make_instance", "sg_encode_instance", "sg_check_instance", "sa_anneal", "sg_sa_anneal_wide",
               "sg_fragment_decimate", "sg_pticm_run", "sg_tn_plan_create", "sg_tn_plan_info_get",
               "sg_tn_plan_destroy", "sg_tn_plan_program", "sg_tn_plan_rounds", "sg_tn_decimate",
               "pt_run", "sg_pt_run_split", "energy", "epsilon"):
        getattr(L, fn).restype = c.c_int
    _lib = L
    return L


def _check(rc: int, what: str) -> None:
    if rc != SG_OK:
        msg = lib().sg_last_error().decode(errors="replace")
        raise SgError(rc, f"{what}: {msg}")


def _np_ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype_name: str):
    if t is None:
        return None
    assert t.is_cuda, f"{dtype_name} tensor must live on the GPU"
    assert t.is_contiguous(), f"{dtype_name} tensor must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------

def make_schedule(kind: int, b0: float, b1: float, S: int) -> np.ndarray:
    out = np.zeros(S, np.float64)
    _check(lib().sg_make_schedule(kind, b0, b1, S, _np_ptr(out)), "sg_make_schedule")
    return out


def make_thresholds(beta, K: int = SG_K_MAX) -> np.ndarray:
    beta = np.ascontiguousarray(beta, np.float64)
    out = np.zeros((len(beta), K), np.uint32)
    _check(lib().sg_make_thresholds(_np_ptr(beta), len(beta), K, _np_ptr(out)), "sg_make_thresholds")
    return out


def make_exchange_thresholds(beta, M: int) -> np.ndarray:
    beta = np.ascontiguousarray(beta, np.float64)
    out = np.zeros((len(beta) - 1, M), np.uint32)
    _check(lib().sg_make_exchange_thresholds(_np_ptr(beta), len(beta), M, _np_ptr(out)),
           "sg_make_exchange_thresholds")
    return out


def exchange_table_width(beta) -> int:
    beta = np.ascontiguousarray(beta, np.float64)
    w = lib().sg_exchange_table_width(_np_ptr(beta), len(beta))
    if w < 1:
        _check(w, "sg_exchange_table_width")
    return int(w)


def make_instance(L: int, cls: int, seed: int):
    """Host generator: returns (J int8 [6][N], planted int8 [N], E_gs)."""
    N = L ** 3
    J = np.zeros((6, N), np.int8)
    g = np.zeros(N, np.int8)
    egs = ctypes.c_int64(0)
    _check(lib().sg_make_instance(L, cls, seed & 0xFFFFFFFFFFFFFFFF, _np_ptr(J), _np_ptr(g),
                                  ctypes.addressof(egs)), "sg_make_instance")
    return J, g, int(egs.value)


def jenc_bytes(L: int) -> int:
    return int(lib().sg_jenc_bytes(L))


# ---------------------------------------------------------------------------
# device-side wrappers
# ---------------------------------------------------------------------------

class Instance:
    """An instance resident on the GPU: couplings J (torch int8 [6][N]),
    optional encoded couplings, E_gs and its chain counter word."""

    def __init__(self, L: int, J, E_gs: int, chain: int = 0, encode: bool | None = None,
                 device="cuda"):
        import torch
        self.L = int(L)
        self.E_gs = int(E_gs)
        self.chain = int(chain)
        if isinstance(J, np.ndarray):
            J = torch.from_numpy(np.ascontiguousarray(J, np.int8))
        self.J = J.to(device).contiguous()
        self.jenc = None
        if encode is None:
            encode = self.L > SG_LDS_MAX_L
        if encode:
            self.jenc = torch.empty(jenc_bytes(self.L) // 4, dtype=torch.int32, device=self.J.device)
            _check(lib().sg_encode_instance(ctypes.byref(self.struct(with_jenc=False)),
                                            _dptr(self.jenc, "jenc"), _stream(None)),
                   "sg_encode_instance")

    @classmethod
    def generate(cls, L: int, seed: int, chain: int = 0, klass: int = 6, **kw):
        J, planted, egs = make_instance(L, klass, seed)
        inst = cls(L, J, egs, chain, **kw)
        inst.planted = planted
        return inst

    def struct(self, with_jenc: bool = True) -> sg_instance:
        s = sg_instance()
        s.L = self.L
        s.J = self.J.data_ptr()
        s.jenc = self.jenc.data_ptr() if (with_jenc and self.jenc is not None) else None
        s.E_gs = self.E_gs
        s.chain = self.chain & 0xFFFFFFFF
        return s


def check_instance(inst: Instance, stream=None) -> int:
    import torch
    st = torch.empty(1, dtype=torch.int32, device=inst.J.device)
    _check(lib().sg_check_instance(ctypes.byref(inst.struct()), _dptr(st, "status"),
                                   _stream(stream)), "sg_check_instance")
    return int(st.item())


def _workspace(L: int, n_rep: int, device):
    """Device scratch: required for lattices whose spins do not fit in LDS
    (L > 32); for few replicas of L > 24 it lets sa_anneal spread the anneal
    over the whole device.  None when neither applies."""
    import torch
    nbytes = max(sa_workspace_bytes(L, n_rep), sa_wide_workspace_bytes(L, n_rep))
    if nbytes == 0:
        return None
    return torch.empty(nbytes // 4, dtype=torch.int32, device=device)


def _with_workspace(args: "sg_sa_args", ws) -> "sg_sa_args":
    if ws is not None:
        args.workspace = ws.data_ptr()
        args.workspace_bytes = ws.numel() * 4
    return args


def sa_anneal(inst: Instance, thr, n_rep: int, seed: int, rep0: int = 0, sweep0: int = 0,
              spins=None, want_emin: bool = False, stream=None, out=None):
    """Anneal n_rep replicas with the threshold rows thr (torch uint32-as-int32
    [n_sweeps][K] on the GPU).  spins=None draws them from the init stream.
    Returns (spins int8 [n_rep][N], energy int32 [n_rep], emin or None)."""
    import torch
    dev = inst.J.device
    N = inst.L ** 3
    S, K = int(thr.shape[0]), int(thr.shape[1])
    init_random = spins is None
    if out is None:
        sp = torch.empty((n_rep, N), dtype=torch.int8, device=dev) if init_random else spins
        en = torch.empty(n_rep, dtype=torch.int32, device=dev)
        em = torch.empty(n_rep, dtype=torch.int32, device=dev) if want_emin else None
    else:
        sp, en, em = out
        if not init_random and sp.data_ptr() != spins.data_ptr():
            sp.copy_(spins)
    args = sg_sa_args(n_rep=n_rep, rep0=rep0, n_sweeps=S, sweep0=sweep0, K=K,
                      init_random=1 if init_random else 0, seed=seed & 0xFFFFFFFFFFFFFFFF)
    ws = _workspace(inst.L, n_rep, dev)
    _with_workspace(args, ws)
    _check(lib().sa_anneal(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                           _dptr(sp, "spins"), _dptr(en, "energy"), _dptr(em, "emin"),
                           _stream(stream)), "sa_anneal")
    return sp, en, em


def pt_run(inst: Instance, thr, thrx, n_runs: int, n_steps: int, seed: int, run0: int = 0,
           step0: int = 0, spins=None, pos=None, want_trace: bool = False,
           want_swaps: bool = False, stream=None, groups: int = 1, waves: int = 0, workspace=None,
           check: bool = True):
    """Parallel tempering.  thr: device [T][K]; thrx: device [T-1][M].
    groups != 1 (or waves != 0) calls sg_pt_run_split: each run spread over
    that many work groups (0: as many as fill the device), same results;
    workspace: a device tensor of at least pt_split_workspace_bytes(n_runs,
    T) bytes, allocated here when None.  pos (with spins) must hold a
    permutation of the slots per run: checked here, SgError(SG_EINVAL).
    check (split form, outside stream capture): wait for the call and raise
    SgError(SG_EBUSY) when a work group gave up waiting on another (the
    results are then invalid); with check=False, or under capture, the
    caller reads the status word itself.
    Returns dict(spins [n_runs][T][N], energy [n_runs][T], pos [n_runs][T],
    emin_trace, swap_acc, and for the split form `workspace`, whose first
    int32 is the status word: 0, bit 0 a group gave up waiting)."""
    import torch
    dev = inst.J.device
    N = inst.L ** 3
    T, K = int(thr.shape[0]), int(thr.shape[1])
    M = int(thrx.shape[1])
    init_random = spins is None
    sp = torch.empty((n_runs, T, N), dtype=torch.int8, device=dev) if init_random else spins
    ps = torch.empty((n_runs, T), dtype=torch.int32, device=dev) if init_random else pos
    if not init_random:
        ident = torch.arange(T, dtype=ps.dtype, device=ps.device)
        if not bool((torch.sort(ps.reshape(n_runs, T), dim=1).values == ident).all()):
            raise SgError(SG_EINVAL, "pt_run: pos is not a permutation of the ladder slots in every run")
    en = torch.empty((n_runs, T), dtype=torch.int32, device=dev)
    tr = torch.empty((n_runs, n_steps), dtype=torch.int32, device=dev) if want_trace else None
    sw = torch.zeros((n_runs, T - 1), dtype=torch.int32, device=dev) if want_swaps else None
    args = sg_pt_args(n_runs=n_runs, run0=run0, T=T, n_steps=n_steps, step0=step0, K=K, M=M,
                      init_random=1 if init_random else 0, seed=seed & 0xFFFFFFFFFFFFFFFF)
    out = {"spins": sp, "energy": en, "pos": ps, "emin_trace": tr, "swap_acc": sw}
    if groups == 1 and waves == 0:
        _check(lib().pt_run(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                            _dptr(thrx, "thrx"), _dptr(sp, "spins"), _dptr(en, "energy"),
                            _dptr(ps, "pos"), _dptr(tr, "emin_trace"), _dptr(sw, "swap_acc"),
                            _stream(stream)), "pt_run")
        return out
    nbytes = pt_split_workspace_bytes(n_runs, T)
    if workspace is None:
        workspace = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=dev)
    _check(lib().sg_pt_run_split(ctypes.byref(inst.struct()), ctypes.byref(args), groups, waves,
                                 _dptr(thr, "thr"), _dptr(thrx, "thrx"), _dptr(sp, "spins"), _dptr(en, "energy"),
                                 _dptr(ps, "pos"), _dptr(tr, "emin_trace"), _dptr(sw, "swap_acc"),
                                 _dptr(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                                 _stream(stream)), "sg_pt_run_split")
    out["workspace"] = workspace
    if check and not torch.cuda.is_current_stream_capturing():
        status = int(workspace.view(torch.int32)[0].item())
        if status & 1:
            raise SgError(SG_EBUSY, "sg_pt_run_split: a work group gave up waiting on another "
                                    "(other work held the device); the results are invalid")
    return out


def pt_split_workspace_bytes(n_runs: int, T: int) -> int:
    n = lib().sg_pt_split_workspace_bytes(n_runs, T)
    if n == 0:
        raise SgError(SG_EINVAL, f"sg_pt_split_workspace_bytes: n_runs = {n_runs}, T = {T}")
    return int(n)


def pticm_run(inst: Instance, thr, thrx, n_runs: int, n_steps: int, seed: int, icm_from: int = 0,
              run0: int = 0, step0: int = 0, spins=None, pos=None, want_trace: bool = False,
              want_swaps: bool = False, want_icm: bool = False, stream=None):
    """Parallel tempering with isoenergetic cluster moves: two copies of the
    T-slot ladder thr (device [T][K]).  Returns dict(spins [n_runs][2T][N],
    energy [n_runs][2T], pos, emin_trace, swap_acc, icm_flipped)."""
    import torch
    dev = inst.J.device
    N = inst.L ** 3
    T, K = int(thr.shape[0]), int(thr.shape[1])
    M = int(thrx.shape[1])
    W = 2 * T
    init_random = spins is None
    sp = torch.empty((n_runs, W, N), dtype=torch.int8, device=dev) if init_random else spins
    ps = torch.empty((n_runs, W), dtype=torch.int32, device=dev) if init_random else pos
    en = torch.empty((n_runs, W), dtype=torch.int32, device=dev)
    tr = torch.empty((n_runs, n_steps), dtype=torch.int32, device=dev) if want_trace else None
    sw = torch.zeros((n_runs, 2 * (T - 1)), dtype=torch.int32, device=dev) if want_swaps else None
    ic = torch.empty((n_runs, n_steps), dtype=torch.int32, device=dev) if want_icm else None
    args = sg_pticm_args(n_runs=n_runs, run0=run0, T=T, n_steps=n_steps, step0=step0, K=K, M=M,
                         init_random=1 if init_random else 0, icm_from=icm_from,
                         seed=seed & 0xFFFFFFFFFFFFFFFF)
    _check(lib().sg_pticm_run(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                              _dptr(thrx, "thrx"), _dptr(sp, "spins"), _dptr(en, "energy"), _dptr(ps, "pos"),
                              _dptr(tr, "emin_trace"), _dptr(sw, "swap_acc"), _dptr(ic, "icm_flipped"),
                              _stream(stream)), "sg_pticm_run")
    return {"spins": sp, "energy": en, "pos": ps, "emin_trace": tr, "swap_acc": sw, "icm_flipped": ic}


def sa_variants(L: int) -> list[dict]:
    buf = (sg_sa_variant * 16)()
    n = lib().sg_sa_variants(L, 16, ctypes.cast(buf, ctypes.c_void_p))
    if n < 0:
        _check(n, "sg_sa_variants")
    return [{"L": buf[i].L, "replicas_per_group": buf[i].replicas_per_group,
             "waves_per_group": buf[i].waves_per_group, "both_encodings": bool(buf[i].both_encodings),
             "couplings_in_hbm": bool(buf[i].couplings_in_hbm), "spins_in_hbm": bool(buf[i].spins_in_hbm),
             "lds_bytes": buf[i].lds_bytes} for i in range(n)]


def sa_workspace_bytes(L: int, n_rep: int) -> int:
    return int(lib().sg_sa_workspace_bytes(L, n_rep))


def sa_wide_workspace_bytes(L: int, n_rep: int) -> int:
    return int(lib().sg_sa_wide_workspace_bytes(L, n_rep))


def sa_anneal_wide(inst: Instance, thr, n_rep: int, seed: int, rep0: int = 0, sweep0: int = 0,
                   spins=None, stream=None):
    """sa_anneal on the multi-work-group path (L = 26..32, 64), whatever
    n_rep is.  Returns (spins, energy); results equal sa_anneal's."""
    import torch
    dev = inst.J.device
    L = inst.L
    N = L ** 3
    S, K = int(thr.shape[0]), int(thr.shape[1])
    init_random = spins is None
    sp = torch.empty((n_rep, N), dtype=torch.int8, device=dev) if init_random else spins
    en = torch.empty(n_rep, dtype=torch.int32, device=dev)
    ws = torch.empty(n_rep * L * L * ((L + 3) // 4), dtype=torch.int32, device=dev)
    args = sg_sa_args(n_rep=n_rep, rep0=rep0, n_sweeps=S, sweep0=sweep0, K=K,
                      init_random=1 if init_random else 0, seed=seed & 0xFFFFFFFFFFFFFFFF)
    _with_workspace(args, ws)
    _check(lib().sg_sa_anneal_wide(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                                   _dptr(sp, "spins"), _dptr(en, "energy"), _stream(stream)), "sg_sa_anneal_wide")
    return sp, en


def select_variant(L: int, variant: int) -> None:
    _check(lib().sg_sa_select_variant(L, variant), "sg_sa_select_variant")


def selected_variant(L: int) -> int:
    v = lib().sg_sa_selected_variant(L)
    if v < 0:
        _check(v, "sg_sa_selected_variant")
    return v


def sa_anneal_variant(inst: Instance, thr, n_rep: int, seed: int, variant: int, rep0: int = 0,
                      sweep0: int = 0, spins=None, want_emin: bool = False, stream=None):
    """sa_anneal with an explicit launch-shape variant (results are identical)."""
    import torch
    dev = inst.J.device
    N = inst.L ** 3
    S, K = int(thr.shape[0]), int(thr.shape[1])
    init_random = spins is None
    sp = torch.empty((n_rep, N), dtype=torch.int8, device=dev) if init_random else spins
    en = torch.empty(n_rep, dtype=torch.int32, device=dev)
    em = torch.empty(n_rep, dtype=torch.int32, device=dev) if want_emin else None
    args = sg_sa_args(n_rep=n_rep, rep0=rep0, n_sweeps=S, sweep0=sweep0, K=K,
                      init_random=1 if init_random else 0, seed=seed & 0xFFFFFFFFFFFFFFFF)
    ws = _workspace(inst.L, n_rep, dev)
    _with_workspace(args, ws)
    _check(lib().sg_sa_anneal_variant(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                                      _dptr(sp, "spins"), _dptr(en, "energy"), _dptr(em, "emin"),
                                      variant, _stream(stream)), "sg_sa_anneal_variant")
    return sp, en, em


def autotune(L: int, n_rep: int = 4096, n_sweeps: int = 32, repeats: int = 3, stream=None) -> dict:
    """Time every launch shape of size L, check they agree bit for bit,
    select the fastest.  Returns {"selected": i, "results": [...]}."""
    buf = (sg_sa_tune_result * 16)()
    r = lib().sg_autotune_sa(L, n_rep, n_sweeps, repeats, ctypes.cast(buf, ctypes.c_void_p), 16,
                             _stream(stream))
    if r < 0:
        _check(r, "sg_autotune_sa")
    nv = len(sa_variants(L))
    return {"selected": int(r), "results": [{"variant": buf[i].variant, "identical": bool(buf[i].identical),
                                              "ms": float(buf[i].ms), "attempts_per_s": buf[i].attempts_per_s}
                                             for i in range(nv)]}


def save_tuning(path: str, Ls) -> None:
    import json
    with open(path, "w") as f:
        json.dump({str(L): selected_variant(L) for L in Ls}, f)


def load_tuning(path: str) -> dict:
    import json
    with open(path) as f:
        choice = {int(k): int(v) for k, v in json.load(f).items()}
    for L, v in choice.items():
        select_variant(L, v)
    return choice


def fragment_decimate(inst: Instance, thr, core: int, halo: int, replicas: int, order: int, n_runs: int,
                      seed: int, run0: int = 0, stream=None):
    """The linear-time meta-heuristic: decimate every core of c^3 spins from
    the best of `replicas` anneals of its (c + 2 halo)^3 fragment, phase by
    phase (order 0 colour classes, 1 diagonal wavefront).  thr: device uint32
    [n_sweeps][K].  Returns (spins int8 [n_runs][N], energy int32 [n_runs])."""
    import torch
    dev = inst.J.device
    N = inst.L ** 3
    S, K = int(thr.shape[0]), int(thr.shape[1])
    sp = torch.empty((n_runs, N), dtype=torch.int8, device=dev)
    en = torch.empty(n_runs, dtype=torch.int32, device=dev)
    args = sg_frag_args(core=core, halo=halo, replicas=replicas, order=order, n_runs=n_runs, run0=run0,
                        n_sweeps=S, K=K, seed=seed & 0xFFFFFFFFFFFFFFFF)
    _check(lib().sg_fragment_decimate(ctypes.byref(inst.struct()), ctypes.byref(args), _dptr(thr, "thr"),
                                      _dptr(sp, "spins"), _dptr(en, "energy"), _stream(stream)),
           "sg_fragment_decimate")
    return sp, en


class TnPlan:
    """Plan of the tensor-network fragment decimation of an L^3 lattice with
    fragment edge 2 halo + 1 in phase order `order` (host work only)."""

    def __init__(self, L: int, halo: int, order: int = 1, lds_max_bits: int = 0):
        h = ctypes.c_void_p()
        _check(lib().sg_tn_plan_create(L, halo, order, lds_max_bits, ctypes.byref(h)), "sg_tn_plan_create")
        self._h = h
        self.L, self.halo, self.order = int(L), int(halo), int(order)

    def info(self) -> dict:
        out = sg_tn_plan_info()
        _check(lib().sg_tn_plan_info_get(self._h, ctypes.byref(out)), "sg_tn_plan_info_get")
        return {name: getattr(out, name) for name, _ in sg_tn_plan_info._fields_}

    def program(self):
        """(shapes [S][4] int32, steps [T][16] int32, items [N][2] int32)."""
        ns, nt, ni = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sg_tn_plan_program(self._h, ctypes.byref(ns), None, ctypes.byref(nt), None,
                                        ctypes.byref(ni), None), "sg_tn_plan_program")
        shapes = np.zeros((ns.value, 4), np.int32)
        steps = np.zeros((max(nt.value, 1), 16), np.int32)
        items = np.zeros((ni.value, 2), np.int32)
        _check(lib().sg_tn_plan_program(self._h, ctypes.byref(ns), _np_ptr(shapes), ctypes.byref(nt),
                                        _np_ptr(steps), ctypes.byref(ni), _np_ptr(items)), "sg_tn_plan_program")
        return shapes, steps[:nt.value], items

    def rounds(self):
        """(shape_rounds [S][2] int32: first round and count per shape,
        rounds [R][4] int32: first step within the shape, fused, read bits,
        slot case of the second step | its rank << 8)."""
        nr = ctypes.c_int32()
        _check(lib().sg_tn_plan_rounds(self._h, ctypes.byref(nr), None, None), "sg_tn_plan_rounds")
        shape_rounds = np.zeros((self.info()["n_shapes"], 2), np.int32)
        rounds = np.zeros((max(nr.value, 1), 4), np.int32)
        _check(lib().sg_tn_plan_rounds(self._h, ctypes.byref(nr), _np_ptr(shape_rounds), _np_ptr(rounds)),
               "sg_tn_plan_rounds")
        return shape_rounds, rounds[:nr.value]

    def workspace_bytes(self, n_inst: int, full: bool = True) -> int:
        n = int(lib().sg_tn_workspace_bytes(self._h, n_inst, 1 if full else 0))
        if n < 0:
            _check(n, "sg_tn_workspace_bytes")
        return n

    def close(self):
        if getattr(self, "_h", None):
            lib().sg_tn_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tn_decimate(plan: TnPlan, J, beta: float = 2.0, tropical: bool = False, want_score: bool = True,
                workspace=None, stream=None):
    """Decimate a batch of instances of the plan's L.  J: device int8
    [n_inst][6][N] (or [6][N], or an Instance).  Returns (spins int8
    [n_inst][N], energy int32 [n_inst], score float64 [n_inst][N] or None)."""
    import torch
    if isinstance(J, Instance):
        J = J.J
    if J.dim() == 2:
        J = J.unsqueeze(0)
    J = J.contiguous()
    n_inst, N = int(J.shape[0]), int(J.shape[2])
    dev = J.device
    sp = torch.empty((n_inst, N), dtype=torch.int8, device=dev)
    en = torch.empty(n_inst, dtype=torch.int32, device=dev)
    sc = torch.empty((n_inst, N), dtype=torch.float64, device=dev) if want_score else None
    if workspace is None:
        # the whole largest phase at once when that is at most 8 GiB, else
        # 8 GiB (or the least that works): the workspace tables then go in passes
        cap = 8 << 30
        nbytes = plan.workspace_bytes(n_inst, full=True)
        if nbytes > cap:
            nbytes = max(cap, plan.workspace_bytes(n_inst, full=False))
        workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    args = sg_tn_args(J=J.data_ptr(), n_inst=n_inst, tropical=1 if tropical else 0, beta=float(beta),
                      spins_out=sp.data_ptr(), score_out=sc.data_ptr() if sc is not None else None,
                      energy_out=en.data_ptr(), workspace=workspace.data_ptr(),
                      workspace_bytes=workspace.numel() * workspace.element_size())
    _check(lib().sg_tn_decimate(plan._h, ctypes.byref(args), _stream(stream)), "sg_tn_decimate")
    return sp, en, sc


def energy(inst: Instance, spins, stream=None):
    import torch
    n = int(spins.shape[0])
    out = torch.empty(n, dtype=torch.int32, device=spins.device)
    _check(lib().energy(ctypes.byref(inst.struct()), n, _dptr(spins, "spins"), _dptr(out, "energy"),
                        _stream(stream)), "energy")
    return out


def epsilon(energy_t, E_gs: int, stream=None):
    import torch
    n = int(energy_t.numel())
    out = torch.empty(n, dtype=torch.float64, device=energy_t.device)
    _check(lib().epsilon(_dptr(energy_t, "energy"), n, int(E_gs), _dptr(out, "eps"),
                         _stream(stream)), "epsilon")
    return out


def epsilon_stats(energy_t, E_gs, targets=(), eps_max: float = 1.0, n_bins: int = 0, stream=None):
    """Per-instance gap statistics on the device (epsilon_stats).  energy_t:
    int32 [n_groups][group_size] (or 1-D: one group); E_gs: an int or a
    sequence of n_groups ints.  Returns device tensors: ``sum`` int64,
    ``emin``, ``emax`` int32, ``n_le`` int32 [n_groups][n_targets] and, with
    n_bins > 0, ``hist`` int32 bits of uint32 counts [n_groups][n_bins]."""
    import torch
    e = energy_t if energy_t.dim() == 2 else energy_t.reshape(1, -1)
    G, n = int(e.shape[0]), int(e.shape[1])
    if isinstance(E_gs, torch.Tensor) and E_gs.is_cuda:
        assert E_gs.dtype == torch.int64 and E_gs.numel() == G
        gs = E_gs.contiguous()
    else:
        gs_host = np.broadcast_to(np.asarray(E_gs, np.int64), (G,))
        gs = torch.from_numpy(np.array(gs_host, np.int64)).to(e.device)
    tg = np.ascontiguousarray(np.asarray(targets, np.float64).reshape(-1))
    raw = torch.empty((G, ctypes.sizeof(sg_eps_stats) // 4), dtype=torch.int32, device=e.device)
    hist = torch.empty((G, n_bins), dtype=torch.int32, device=e.device) if n_bins > 0 else None
    _check(lib().epsilon_stats(_dptr(e, "energy"), G, n, _dptr(gs, "E_gs"),
                               ctypes.c_void_p(tg.ctypes.data) if tg.size else None, int(tg.size),
                               float(eps_max), int(n_bins), _dptr(raw, "stats"), _dptr(hist, "hist"),
                               _stream(stream)), "epsilon_stats")
    out = {"sum": raw[:, 0:2].contiguous().view(torch.int64).reshape(G), "emin": raw[:, 2], "emax": raw[:, 3],
           "n_le": raw[:, 5:5 + tg.size], "n": n}
    if hist is not None:
        out["hist"] = hist
    return out


def mean_epsilon(stats: dict, E_gs) -> np.ndarray:
    """Mean gap per group from the exact energy sums of epsilon_stats (host
    NumPy, one division per group): (sum - n E_gs) / (n |E_gs|)."""
    s = stats["sum"].cpu().numpy().astype(np.int64)
    n = int(stats["n"])
    if hasattr(E_gs, "cpu"):
        E_gs = E_gs.cpu().numpy()
    gs = np.broadcast_to(np.asarray(E_gs, np.int64), s.shape)
    return (s - n * gs).astype(np.float64) / (n * np.abs(gs).astype(np.float64))


def to_device_u32(a: np.ndarray, device="cuda"):
    """Upload a uint32 table (stored as int32 bits) to the GPU."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(device)


SG_BATCH_GRAPH = 1


class SAJob:
    """One sa_anneal call described for a batch: the instance, its replica
    range and schedule, and the output buffers (allocated here)."""

    def __init__(self, inst: Instance, thr, n_rep: int, seed: int, rep0: int = 0, sweep0: int = 0,
                 spins=None, want_emin: bool = False, energy=None):
        """energy: an int32 device tensor of n_rep entries (e.g. a row of a
        shared [jobs][n_rep] array for epsilon_stats) to receive the final
        energies; allocated here when None."""
        import torch
        dev = inst.J.device
        self.inst, self.thr, self.n_rep = inst, thr, n_rep
        self.seed, self.rep0, self.sweep0 = seed, rep0, sweep0
        self.init_random = spins is None
        self.spins = torch.empty((n_rep, inst.L ** 3), dtype=torch.int8, device=dev) if spins is None else spins
        if energy is not None:
            assert energy.dtype == torch.int32 and energy.numel() == n_rep and energy.is_contiguous()
        self.energy = torch.empty(n_rep, dtype=torch.int32, device=dev) if energy is None else energy
        self.emin = torch.empty(n_rep, dtype=torch.int32, device=dev) if want_emin else None
        self.workspace = _workspace(inst.L, n_rep, dev)

    def struct(self) -> sg_sa_job:
        j = sg_sa_job()
        j.inst = self.inst.struct()
        j.args = sg_sa_args(n_rep=self.n_rep, rep0=self.rep0, n_sweeps=int(self.thr.shape[0]),
                            sweep0=self.sweep0, K=int(self.thr.shape[1]),
                            init_random=1 if self.init_random else 0,
                            seed=self.seed & 0xFFFFFFFFFFFFFFFF)
        _with_workspace(j.args, self.workspace)
        j.thr = self.thr.data_ptr()
        j.spins = self.spins.data_ptr()
        j.energy = self.energy.data_ptr()
        j.emin = self.emin.data_ptr() if self.emin is not None else None
        return j


class Batch:
    """A batched annealing plan (sg_batch_*): jobs grouped by L, one kernel
    per L on parallel branches, optionally replayed as a hipGraph."""

    def __init__(self, jobs: list, graph: bool = True):
        self.jobs = list(jobs)   # keeps the device buffers alive
        arr = (sg_sa_job * len(self.jobs))(*[j.struct() for j in self.jobs])
        h = ctypes.c_void_p()
        _check(lib().sg_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(self.jobs),
                                     SG_BATCH_GRAPH if graph else 0, ctypes.byref(h)), "sg_batch_create")
        self.handle = h

    def launch(self, stream=None):
        _check(lib().sg_batch_launch(self.handle, _stream(stream)), "sg_batch_launch")

    def info(self):
        nk = ctypes.c_int32()
        ng = ctypes.c_int64()
        att = ctypes.c_double()
        _check(lib().sg_batch_info(self.handle, ctypes.byref(nk), ctypes.byref(ng), ctypes.byref(att)),
               "sg_batch_info")
        return {"kernels": nk.value, "groups": ng.value, "attempts": att.value}

    def kernels(self):
        n = 64
        Ls = np.zeros(n, np.int32)
        att = np.zeros(n, np.float64)
        ms = np.zeros(n, np.float32)
        m = lib().sg_batch_kernels(self.handle, n, _np_ptr(Ls), _np_ptr(att), _np_ptr(ms))
        return [{"L": int(Ls[i]), "attempts": float(att[i]), "ms": float(ms[i])} for i in range(m)]

    def close(self):
        if self.handle:
            lib().sg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
