"""ctypes view of the plain C oracle (``oracle/oracle.c``).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it and shares no code with it.

Every wrapper returns NumPy arrays; all arithmetic happens in the C file.
The tensor-network fragment oracle is plain NumPy, in ``oracle/tn.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so (plain C99, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        c = ctypes
        L.orc_site.restype = c.c_int64
        L.orc_site.argtypes = [c.c_int] * 6
        L.orc_nbr.restype = c.c_int64
        L.orc_nbr.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int64, c.c_int]
        L.orc_sm64_next.restype = c.c_uint64
        L.orc_sm64_next.argtypes = [c.POINTER(c.c_uint64)]
        L.orc_philox.restype = None
        L.orc_philox.argtypes = [u32p, c.c_uint32, c.c_uint32, u32p]
        L.orc_make_instance.restype = c.c_int
        L.orc_make_instance.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                        i8p, i8p, c.POINTER(c.c_int64)]
        L.orc_energy.restype = c.c_int64
        L.orc_energy.argtypes = [c.c_int, c.c_int, c.c_int, i8p, i8p]
        L.orc_local_field.restype = c.c_int64
        L.orc_local_field.argtypes = [c.c_int, c.c_int, c.c_int, i8p, i8p, c.c_int64]
        L.orc_epsilon.restype = c.c_double
        L.orc_epsilon.argtypes = [c.c_int64, c.c_int64]
        L.orc_eps_stats.restype = c.c_int
        L.orc_eps_stats.argtypes = [i32p, c.c_int, c.c_int, i64p, f64p, c.c_int, c.c_double, c.c_int,
                                    i64p, i32p, i32p, i32p, c.c_void_p]
        L.orc_schedule.restype = c.c_int
        L.orc_schedule.argtypes = [c.c_int, c.c_double, c.c_double, c.c_int, f64p]
        L.orc_thresholds.restype = c.c_int
        L.orc_thresholds.argtypes = [f64p, c.c_int, c.c_int, u32p]
        L.orc_exchange_thresholds.restype = c.c_int
        L.orc_exchange_thresholds.argtypes = [f64p, c.c_int, c.c_int, u32p]
        L.orc_sa_run.restype = c.c_int
        L.orc_sa_run.argtypes = [c.c_int, i8p, c.c_uint64, c.c_uint32, c.c_uint32, c.c_int,
                                 u32p, c.c_int, c.c_int, c.c_int, c.c_int,
                                 i8p, i64p, c.c_void_p, c.c_int]
        L.orc_sa_run_reversed.restype = c.c_int
        L.orc_sa_run_reversed.argtypes = [c.c_int, i8p, c.c_uint64, c.c_uint32, c.c_uint32,
                                          c.c_int, u32p, c.c_int, c.c_int, c.c_int, c.c_int,
                                          i8p, i64p]
        L.orc_pt_run.restype = c.c_int
        L.orc_pt_run.argtypes = [c.c_int, i8p, c.c_uint64, c.c_uint32, c.c_int,
                                 u32p, c.c_int, u32p, c.c_int, c.c_int, c.c_int, c.c_int,
                                 i8p, i64p, i32p, c.c_void_p, c.c_void_p, c.c_int]
        L.orc_init_spins.restype = None
        L.orc_init_spins.argtypes = [c.c_int, c.c_uint64, c.c_uint32, c.c_uint32, i8p]
        L.orc_metropolis_uniform.restype = c.c_uint32
        L.orc_metropolis_uniform.argtypes = [c.c_int, c.c_uint64, c.c_uint32, c.c_uint32,
                                             c.c_int, c.c_int64]
        L.orc_pticm_run.restype = c.c_int
        L.orc_pticm_run.argtypes = [c.c_int, i8p, c.c_uint64, c.c_uint32, c.c_int,
                                    u32p, c.c_int, u32p, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                    i8p, i64p, i32p, c.c_void_p, c.c_void_p, c.c_void_p, c.c_int]
        L.orc_icm_move.restype = c.c_int64
        L.orc_icm_move.argtypes = [c.c_int, i8p, i8p, i8p, c.c_uint32]
        for fn in ("orc_frag_decimate", "orc_frag_decimate_reversed"):
            getattr(L, fn).restype = c.c_int
            getattr(L, fn).argtypes = [c.c_int, i8p, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                       c.c_uint32, u32p, c.c_int, c.c_int, i8p]
        L.orc_frag_anneal.restype = c.c_int
        L.orc_frag_anneal.argtypes = [c.c_int, i8p, c.c_int, c.c_int, c.c_int64, c.c_int, c.c_uint64,
                                      c.c_uint32, u32p, c.c_int, c.c_int, i8p, i8p,
                                      c.POINTER(c.c_int64)]
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def philox(ctr, key0: int, key1: int) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    lib().orc_philox(c, key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF, out)
    return out


def sm64_stream(state: int, n: int) -> list[int]:
    st = ctypes.c_uint64(state & 0xFFFFFFFFFFFFFFFF)
    return [lib().orc_sm64_next(ctypes.byref(st)) for _ in range(n)]


def make_instance(L: int, cls: int, seed: int, dims=None, periodic: bool = True):
    """Return (J [6][N] int8, planted [N] int8, E_gs int)."""
    Lx, Ly, Lz = dims if dims is not None else (L, L, L)
    N = Lx * Ly * Lz
    J = np.zeros(6 * N, np.int8)
    g = np.zeros(N, np.int8)
    egs = ctypes.c_int64(0)
    _check(lib().orc_make_instance(Lx, Ly, Lz, 1 if periodic else 0, cls,
                                   seed & 0xFFFFFFFFFFFFFFFF, J, g, ctypes.byref(egs)),
           "make_instance")
    return J.reshape(6, N), g, int(egs.value)


def energy(J: np.ndarray, s: np.ndarray, dims) -> int:
    Lx, Ly, Lz = dims
    return int(lib().orc_energy(Lx, Ly, Lz, np.ascontiguousarray(J, np.int8).reshape(-1),
                                np.ascontiguousarray(s, np.int8).reshape(-1)))


def local_field(J, s, dims, i: int) -> int:
    Lx, Ly, Lz = dims
    return int(lib().orc_local_field(Lx, Ly, Lz, np.ascontiguousarray(J, np.int8).reshape(-1),
                                     np.ascontiguousarray(s, np.int8).reshape(-1), i))


def epsilon(E: int, E_gs: int) -> float:
    return float(lib().orc_epsilon(int(E), int(E_gs)))


def eps_stats(energy, E_gs, targets=(), eps_max: float = 1.0, n_bins: int = 0):
    """Per-group optimality-gap statistics (orc_eps_stats).  energy: int32
    [n_groups][group_size]; E_gs: one value per group.  Returns a dict of
    NumPy arrays: sum, emin, emax, n_le [n_groups][n_targets] and, when
    n_bins > 0, hist [n_groups][n_bins]."""
    e = np.ascontiguousarray(energy, np.int32)
    if e.ndim == 1:
        e = e[None, :]
    G, n = e.shape
    gs = np.ascontiguousarray(np.broadcast_to(np.asarray(E_gs, np.int64), (G,)))
    tg = np.ascontiguousarray(np.asarray(targets, np.float64).reshape(-1))
    if tg.size == 0:
        tg_arr = np.zeros(1, np.float64)
    else:
        tg_arr = tg
    out = {"sum": np.zeros(G, np.int64), "emin": np.zeros(G, np.int32), "emax": np.zeros(G, np.int32),
           "n_le": np.zeros((G, max(1, tg.size)), np.int32)}
    hist = np.zeros((G, n_bins), np.uint32) if n_bins > 0 else None
    _check(lib().orc_eps_stats(e, G, n, gs, tg_arr, int(tg.size), float(eps_max), int(n_bins),
                               out["sum"], out["emin"], out["emax"], out["n_le"],
                               hist.ctypes.data if hist is not None else None), "orc_eps_stats")
    out["n_le"] = out["n_le"][:, :tg.size]
    if hist is not None:
        out["hist"] = hist
    return out


def schedule(kind: int, b0: float, b1: float, S: int) -> np.ndarray:
    out = np.zeros(S, np.float64)
    _check(lib().orc_schedule(kind, b0, b1, S, out), "schedule")
    return out


def thresholds(beta: np.ndarray, K: int) -> np.ndarray:
    beta = np.ascontiguousarray(beta, np.float64)
    out = np.zeros(len(beta) * K, np.uint32)
    _check(lib().orc_thresholds(beta, len(beta), K, out), "thresholds")
    return out.reshape(len(beta), K)


def exchange_thresholds(beta: np.ndarray, M: int) -> np.ndarray:
    beta = np.ascontiguousarray(beta, np.float64)
    T = len(beta)
    out = np.zeros((T - 1) * M, np.uint32)
    _check(lib().orc_exchange_thresholds(beta, T, M, out), "exchange_thresholds")
    return out.reshape(T - 1, M)


def init_spins(L: int, seed: int, chain: int, replica: int) -> np.ndarray:
    s = np.zeros(L ** 3, np.int8)
    lib().orc_init_spins(L, seed & 0xFFFFFFFFFFFFFFFF, chain, replica, s)
    return s


def metropolis_uniform(L, seed, chain, replica, sweep, i) -> int:
    return int(lib().orc_metropolis_uniform(L, seed & 0xFFFFFFFFFFFFFFFF, chain, replica,
                                            sweep, i))


def sa_run(L, J, seed, chain, thr, n_rep=1, rep0=0, sweep0=0, spins=None, want_emin=False,
           check=False, reversed_order=False):
    """Run n_rep replicas; returns (spins [n_rep][N], energy [n_rep], emin or None)."""
    N = L ** 3
    thr = np.ascontiguousarray(thr, np.uint32)
    S, K = thr.shape
    init_random = spins is None
    sp = np.zeros((n_rep, N), np.int8) if init_random else np.array(spins, np.int8).reshape(n_rep, N)
    sp = np.ascontiguousarray(sp)
    en = np.zeros(n_rep, np.int64)
    Jf = np.ascontiguousarray(J, np.int8).reshape(-1)
    if reversed_order:
        _check(lib().orc_sa_run_reversed(L, Jf, seed & 0xFFFFFFFFFFFFFFFF, chain, rep0, n_rep,
                                         thr.reshape(-1), K, S, sweep0, 1 if init_random else 0,
                                         sp.reshape(-1), en), "sa_run_reversed")
        return sp, en, None
    em = np.zeros(n_rep, np.int64) if want_emin else None
    _check(lib().orc_sa_run(L, Jf, seed & 0xFFFFFFFFFFFFFFFF, chain, rep0, n_rep,
                            thr.reshape(-1), K, S, sweep0, 1 if init_random else 0,
                            sp.reshape(-1), en,
                            em.ctypes.data if em is not None else None, 1 if check else 0),
           "sa_run")
    return sp, en, em


def pt_run(L, J, seed, run, thr, thrx, n_steps, step0=0, spins=None, pos=None,
           want_trace=False, want_swaps=False, check=False):
    """One PT run of T walkers.  Returns dict(spins, energy, pos, emin_trace, swap_acc)."""
    N = L ** 3
    thr = np.ascontiguousarray(thr, np.uint32)
    thrx = np.ascontiguousarray(thrx, np.uint32)
    T, K = thr.shape
    M = thrx.shape[1]
    init_random = spins is None
    sp = np.zeros((T, N), np.int8) if init_random else np.array(spins, np.int8).reshape(T, N)
    sp = np.ascontiguousarray(sp)
    ps = np.arange(T, dtype=np.int32) if pos is None else np.array(pos, np.int32)
    ps = np.ascontiguousarray(ps)
    en = np.zeros(T, np.int64)
    tr = np.zeros(n_steps, np.int64) if want_trace else None
    sw = np.zeros(T - 1, np.uint32) if want_swaps else None
    _check(lib().orc_pt_run(L, np.ascontiguousarray(J, np.int8).reshape(-1),
                            seed & 0xFFFFFFFFFFFFFFFF, run, T, thr.reshape(-1), K,
                            thrx.reshape(-1), M, n_steps, step0, 1 if init_random else 0,
                            sp.reshape(-1), en, ps,
                            tr.ctypes.data if tr is not None else None,
                            sw.ctypes.data if sw is not None else None,
                            1 if check else 0), "pt_run")
    return {"spins": sp, "energy": en, "pos": ps, "emin_trace": tr, "swap_acc": sw}


def frag_decimate(L, J, core, halo, R, seed, run, thr, order=1, reversed_order=False) -> np.ndarray:
    """Fragment decimation (the linear-time meta-heuristic with fixed-sweep SA
    on fragments, R anneals per fragment); returns the decimated
    configuration int8 [N]."""
    thr = np.ascontiguousarray(thr, np.uint32)
    S, K = thr.shape
    dec = np.zeros(L ** 3, np.int8)
    fn = lib().orc_frag_decimate_reversed if reversed_order else lib().orc_frag_decimate
    _check(fn(L, np.ascontiguousarray(J, np.int8).reshape(-1), core, halo, R, order, seed & 0xFFFFFFFFFFFFFFFF,
              run, thr.reshape(-1), K, S, dec), "frag_decimate")
    return dec


def frag_anneal(L, J, core, halo, k, rep, seed, run, thr, dec):
    """Anneal rep of core k with decimation state dec (0 = free); returns
    (fragment spins int8 [l^3], in-fragment energy)."""
    thr = np.ascontiguousarray(thr, np.uint32)
    S, K = thr.shape
    l = core + 2 * halo
    frag = np.zeros(l ** 3, np.int8)
    E = ctypes.c_int64(0)
    _check(lib().orc_frag_anneal(L, np.ascontiguousarray(J, np.int8).reshape(-1), core, halo, k, rep,
                                 seed & 0xFFFFFFFFFFFFFFFF, run, thr.reshape(-1), K, S,
                                 np.ascontiguousarray(dec, np.int8).reshape(-1), frag, ctypes.byref(E)),
           "frag_anneal")
    return frag, int(E.value)


def pticm_run(L, J, seed, run, thr, thrx, n_steps, icm_from=0, step0=0, spins=None, pos=None,
              want_trace=False, want_swaps=False, want_icm=False, check=False):
    """PT with isoenergetic cluster moves: two copies of the T-slot ladder
    (2T walkers).  Returns dict(spins [2T][N], energy, pos, emin_trace,
    swap_acc [2(T-1)], icm_flipped)."""
    N = L ** 3
    thr = np.ascontiguousarray(thr, np.uint32)
    thrx = np.ascontiguousarray(thrx, np.uint32)
    T, K = thr.shape
    M = thrx.shape[1]
    W = 2 * T
    init_random = spins is None
    sp = np.zeros((W, N), np.int8) if init_random else np.array(spins, np.int8).reshape(W, N)
    sp = np.ascontiguousarray(sp)
    ps = np.arange(W, dtype=np.int32) % T if pos is None else np.array(pos, np.int32)
    ps = np.ascontiguousarray(ps)
    en = np.zeros(W, np.int64)
    tr = np.zeros(n_steps, np.int64) if want_trace else None
    sw = np.zeros(2 * (T - 1), np.uint32) if want_swaps else None
    ic = np.zeros(n_steps, np.int64) if want_icm else None
    _check(lib().orc_pticm_run(L, np.ascontiguousarray(J, np.int8).reshape(-1),
                               seed & 0xFFFFFFFFFFFFFFFF, run, T, thr.reshape(-1), K,
                               thrx.reshape(-1), M, n_steps, step0, icm_from, 1 if init_random else 0,
                               sp.reshape(-1), en, ps,
                               tr.ctypes.data if tr is not None else None,
                               sw.ctypes.data if sw is not None else None,
                               ic.ctypes.data if ic is not None else None,
                               1 if check else 0), "pticm_run")
    return {"spins": sp, "energy": en, "pos": ps, "emin_trace": tr, "swap_acc": sw, "icm_flipped": ic}


def icm_move(L, J, sa, sb, u):
    """One cluster move on copies of sa, sb; returns (sa', sb', cluster size)."""
    a = np.ascontiguousarray(np.array(sa, np.int8).reshape(-1))
    b = np.ascontiguousarray(np.array(sb, np.int8).reshape(-1))
    n = lib().orc_icm_move(L, np.ascontiguousarray(J, np.int8).reshape(-1), a, b, u)
    if n < 0:
        raise RuntimeError("oracle icm_move failed")
    return a, b, int(n)
