"""Binding of the anneal server (sg_server_*) and the Poisson serving benchmark.

The server itself is native (csrc/server.hip: scheduler thread, admission,
per-size lanes, chunked continuous batching); this module marshals requests
and measures latency and throughput of a seeded Poisson request stream.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import Instance, _check, _dptr, _np_ptr, lib, make_schedule, make_thresholds, sg_instance, \
    to_device_u32

SG_REQ_QUEUED, SG_REQ_ACTIVE, SG_REQ_DONE, SG_REQ_CANCELLED, SG_REQ_FAILED = range(5)


class sg_server_config(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("chunk_sweeps", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("large_slots", ctypes.c_int32),
                ("skip_age_ms", ctypes.c_int32), ("chunk_attempts", ctypes.c_int64)]


class sg_request(ctypes.Structure):
    _fields_ = [("inst", sg_instance), ("thr", ctypes.c_void_p), ("n_sweeps", ctypes.c_int32),
                ("K", ctypes.c_int32), ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
                ("init_random", ctypes.c_int32), ("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("t_arrival", ctypes.c_double)]


class sg_request_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("done_sweeps", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class sg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("active", ctypes.c_int64), ("queued", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("attempts_completed", ctypes.c_double), ("memory_in_use", ctypes.c_int64)]


_ready = False


def _lib():
    global _ready
    L = lib()
    if not _ready:
        c = ctypes
        vp = c.c_void_p
        L.sg_server_create.argtypes = [c.POINTER(sg_server_config), c.POINTER(vp)]
        L.sg_server_now.argtypes = [vp]
        L.sg_server_now.restype = c.c_double
        L.sg_server_submit.argtypes = [vp, c.POINTER(sg_request), c.POINTER(c.c_uint64)]
        L.sg_server_poll.argtypes = [vp, c.c_uint64, c.POINTER(sg_request_status)]
        L.sg_server_cancel.argtypes = [vp, c.c_uint64]
        L.sg_server_release.argtypes = [vp, c.c_uint64]
        L.sg_server_get_stats.argtypes = [vp, c.POINTER(sg_server_stats)]
        L.sg_server_wait.argtypes = [vp, c.c_double]
        L.sg_server_destroy.argtypes = [vp]
        for fn in ("sg_server_create", "sg_server_submit", "sg_server_poll", "sg_server_cancel", "sg_server_release",
                   "sg_server_get_stats", "sg_server_wait", "sg_server_destroy"):
            getattr(L, fn).restype = c.c_int
        _ready = True
    return L


class Server:
    """A running anneal server on the current device."""

    def __init__(self, max_active=4096, chunk_sweeps=64, memory_budget=8 << 30, large_slots=64,
                 chunk_attempts=0, skip_age_ms=0):
        cfg = sg_server_config(max_active=max_active, chunk_sweeps=chunk_sweeps,
                               memory_budget=memory_budget, large_slots=large_slots,
                               chunk_attempts=chunk_attempts, skip_age_ms=skip_age_ms)
        h = ctypes.c_void_p()
        _check(_lib().sg_server_create(ctypes.byref(cfg), ctypes.byref(h)), "sg_server_create")
        self.h = h
        self._keep = {}

    def now(self) -> float:
        return float(_lib().sg_server_now(self.h))

    def submit(self, inst: Instance, thr, seed: int, replica: int, spins, energy, t_arrival=None,
               init_random=True) -> int:
        r = sg_request()
        r.inst = inst.struct()
        r.thr = thr.data_ptr()
        r.n_sweeps = int(thr.shape[0])
        r.K = int(thr.shape[1])
        r.seed = seed & 0xFFFFFFFFFFFFFFFF
        r.replica = replica & 0xFFFFFFFF
        r.init_random = 1 if init_random else 0
        r.spins = spins.data_ptr()
        r.energy = energy.data_ptr()
        r.t_arrival = self.now() if t_arrival is None else t_arrival
        rid = ctypes.c_uint64()
        _check(_lib().sg_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)), "sg_server_submit")
        self._keep[rid.value] = (inst, thr, spins, energy)
        return rid.value

    def poll(self, rid: int) -> dict:
        st = sg_request_status()
        _check(_lib().sg_server_poll(self.h, rid, ctypes.byref(st)), "sg_server_poll")
        return {"state": st.state, "done_sweeps": st.done_sweeps, "t_arrival": st.t_arrival,
                "t_admit": st.t_admit, "t_done": st.t_done}

    def cancel(self, rid: int) -> None:
        _check(_lib().sg_server_cancel(self.h, rid), "sg_server_cancel")

    def release(self, rid: int) -> None:
        """Forget a finished request (its buffers are no longer borrowed)."""
        _check(_lib().sg_server_release(self.h, rid), "sg_server_release")
        self._keep.pop(rid, None)

    def stats(self) -> dict:
        st = sg_server_stats()
        _check(_lib().sg_server_get_stats(self.h, ctypes.byref(st)), "sg_server_get_stats")
        return {f: getattr(st, f) for f, _ in sg_server_stats._fields_}

    def wait(self, timeout_s: float = 60.0) -> None:
        _check(_lib().sg_server_wait(self.h, timeout_s), "sg_server_wait")

    def close(self) -> None:
        if self.h:
            _lib().sg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Poisson serving benchmark
# ---------------------------------------------------------------------------

SMALL_SIZES = tuple(range(8, 33, 2))   # even L in [8, 32]
LARGE_SIZE = 64


def sweep_grid(lo=64, hi=4096, levels=64):
    """Log-uniform sweep budgets on a grid of `levels` values from lo to hi."""
    return sorted({int(round(lo * (hi / lo) ** (k / (levels - 1)))) for k in range(levels)})


def make_stream(rate, duration, seed, p_large=0.05, pool=4, grid=None):
    """Seeded request stream: arrival offsets (exponential gaps), sizes,
    instance indices in the per-size pool, sweep budgets."""
    rng = np.random.default_rng(seed)
    grid = grid or sweep_grid()
    n = int(rate * duration * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    t = t[t < duration]
    n = len(t)
    large = rng.random(n) < p_large
    L = np.where(large, LARGE_SIZE, rng.choice(SMALL_SIZES, n))
    k = rng.integers(0, pool, n)
    S = np.array(grid)[rng.integers(0, len(grid), n)]
    return {"t": t, "L": L.astype(int), "k": k.astype(int), "S": S.astype(int)}


def run_poisson(torch, rate=2000.0, duration=60.0, warmup=5.0, seed=0x5E7E, pool=4, chunk=512,
                chunk_attempts=1 << 24, p_large=0.05, plain_sample=64, check_sample=32, log=print,
                instance_seed=None, return_requests=False):
    """Drive a server with a Poisson stream; return latency and throughput.
    return_requests: also return, under "requests_detail", the stream, the
    instances, tables and the served spins/energies (for checks; not JSON)."""
    from . import epsilon_stats, mean_epsilon, sa_anneal
    from . import workloads as wl
    total = warmup + duration
    stream = make_stream(rate, total, seed, p_large=p_large, pool=pool)
    n = len(stream["t"])
    sizes = sorted(set(stream["L"].tolist()))
    t0 = time.perf_counter()
    insts = {}
    for L in sizes:
        for k in range(pool):
            s = instance_seed(L, k) if instance_seed else wl.mix64((seed << 8) + L * 131 + k)
            insts[(L, k)] = Instance.generate(L, s, chain=L * 1000 + k)
    grid = sorted(set(stream["S"].tolist()))
    thr = {S: to_device_u32(make_thresholds(make_schedule(0, 0.1, 3.0, S))) for S in grid}
    # one spin buffer for the whole stream, 256-byte aligned slices
    N = np.array([L ** 3 for L in stream["L"]], np.int64)
    off = np.concatenate([[0], np.cumsum((N + 255) // 256 * 256)])
    spins = torch.empty(int(off[-1]), dtype=torch.int8, device="cuda")
    energy = torch.zeros(n, dtype=torch.int32, device="cuda")
    t_setup = time.perf_counter() - t0
    log(f"serve: {n} requests over {total:.0f} s, sizes {sizes}, set-up {t_setup:.1f} s")
    srv = Server(max_active=8192, chunk_sweeps=chunk, large_slots=256, chunk_attempts=chunk_attempts)
    key = wl.philox_seed("serve")
    ids = []
    base = srv.now() + 0.2
    for i in range(n):
        target = base + stream["t"][i]
        while True:
            dt = target - srv.now()
            if dt <= 0:
                break
            if dt > 0.002:
                time.sleep(dt - 0.001)
        inst = insts[(int(stream["L"][i]), int(stream["k"][i]))]
        sp = spins[int(off[i]):int(off[i]) + int(N[i])]
        ids.append(srv.submit(inst, thr[int(stream["S"][i])], key, i, sp, energy[i:i + 1], t_arrival=target))
        if i % 20000 == 0:
            log(f"serve: submitted {i}/{n}, stats {srv.stats()}")
    srv.wait(timeout_s=600.0)
    end = srv.now()
    st = [srv.poll(r) for r in ids]
    for r in ids:
        srv.release(r)
    stats = srv.stats()
    srv.close()
    arrive = np.array([s["t_arrival"] for s in st])
    done = np.array([s["t_done"] for s in st])
    admit = np.array([s["t_admit"] for s in st])
    ok = np.array([s["state"] == SG_REQ_DONE for s in st])
    meas = ok & (arrive - base >= warmup)
    lat = (done - arrive)[meas] * 1e3
    wait_ms = (admit - arrive)[meas] * 1e3
    att = (N * stream["S"]).astype(np.float64)
    span = done[meas].max() - (base + warmup)
    # optimality gap of every served request (Eq. 2, on the device: one
    # group of one trial per request)
    en = energy.cpu().numpy().astype(np.int64)
    egs = np.array([insts[(int(L), int(k))].E_gs for L, k in zip(stream["L"], stream["k"])], np.int64)
    eps = mean_epsilon(epsilon_stats(energy.view(n, 1), egs), egs)
    by_class = {}
    for name, mask in (("small", stream["L"] != LARGE_SIZE), ("large", stream["L"] == LARGE_SIZE)):
        m = meas & mask
        if m.any():
            by_class[name] = {"requests": int(m.sum()), "p50_ms": float(np.percentile((done - arrive)[m] * 1e3, 50)),
                              "p99_ms": float(np.percentile((done - arrive)[m] * 1e3, 99)),
                              "eps_mean": float(eps[m].mean())}
    # the same requests alone, in one sa_anneal call each: identical results
    ident = True
    for i in range(0, n, max(1, n // check_sample)):
        inst = insts[(int(stream["L"][i]), int(stream["k"][i]))]
        sp, e, _ = sa_anneal(inst, thr[int(stream["S"][i])], 1, key, rep0=i)
        torch.cuda.synchronize()
        ident &= bool(torch.equal(sp[0], spins[int(off[i]):int(off[i]) + int(N[i])])) and \
            int(e[0]) == int(en[i])
    # plain form: requests one after another, one sa_anneal call each
    sample = list(range(0, n, max(1, n // plain_sample)))[:plain_sample]
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in sample:
        inst = insts[(int(stream["L"][i]), int(stream["k"][i]))]
        sa_anneal(inst, thr[int(stream["S"][i])], 1, key, rep0=i)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - p0
    plain_rate = float(att[sample].sum() / plain_s)
    served_rate = float(att[meas].sum() / span)
    out = {
        "metric": "served anneal requests (Poisson stream)", "rate_req_s": rate, "duration_s": duration,
        "warmup_s": warmup, "requests": int(meas.sum()), "completed_all": int(ok.sum()), "submitted": n,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()), "admission_wait_p99_ms": float(np.percentile(wait_ms, 99)),
        "attempts_per_s": served_rate, "offered_attempts_per_s": float(att[meas].sum() / duration),
        "plain_sequential_attempts_per_s": plain_rate, "served_over_plain": served_rate / plain_rate,
        "served_equals_alone": ident, "eps_mean": float(eps[meas].mean()),
        "eps_frac_le_1pct": float((eps[meas] <= 0.01).mean()), "by_class": by_class,
        "chunk_sweeps_max": chunk, "chunk_attempts": chunk_attempts,
        "kernel_launches": stats["launches"], "set_up_s": t_setup,
        "drain_s": float(end - (base + total)),
    }
    if return_requests:
        out["requests_detail"] = {"stream": stream, "off": off, "N": N, "spins": spins, "energy": energy,
                                  "key": key, "insts": insts, "thr": thr}
    return out
