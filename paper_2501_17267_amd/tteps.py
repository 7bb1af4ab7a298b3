"""Time-to-epsilon (TTeps) versus system size, in the form of App. D.

For each lattice size L: n_inst instances, n_trials independent annealing
runs (one read each) per instance; the sweep count S walks a grid of powers
of sqrt(2); an instance reaches a target eps at the smallest S whose mean eps
over its trials is at or below the target (Eq. 2; App. D's criterion).  Its
TTeps is the time of one trial at that S, measured three ways:

  plain    one sa_anneal call with one replica (launch to completion)
  batched  all trials of all instances of the size in one batched launch,
           divided by the number of trials in it
  served   mean latency of those trials submitted together to the server

The results at one S are identical across the three forms (same counters),
so they compare at equal eps.  TTeps(L) is the mean over instances; a fit
TTeps = a N^alpha + b (N = L^3, App. D) gives the scaling exponent alpha.
Sizes whose instances do not all reach a target by S_max are reported as
censored for that target.
"""
from __future__ import annotations

import time

import numpy as np

from . import Batch, Instance, SAJob, epsilon, make_schedule, make_thresholds, sa_anneal, to_device_u32
from . import workloads as wl


def sweep_grid(lo=16, hi=32768):
    out, k = [], 0
    while True:
        s = int(round(lo * 2 ** (k / 2)))
        if s > hi:
            return out
        out.append(s)
        k += 1


def _thr(cache, S, schedule=(0, 0.1, 3.0)):
    key = (S,) + tuple(schedule)
    if key not in cache:
        kind, b0, b1 = schedule
        cache[key] = to_device_u32(make_thresholds(make_schedule(kind, b0, b1, S)))
    return cache[key]


def run(torch, sizes=(8, 12, 16, 20, 24, 32, 64), n_inst=20, n_trials=20, targets=(0.01, 0.03, 0.04, 0.05),
        s_max=32768, log=print, served=True, plain_inst=5, schedule=(0, 0.1, 3.0)):
    """schedule: (kind, beta0, beta1) of every anneal (0 linear, 1 geometric)."""
    seed = wl.philox_seed("serve") ^ 0x77
    thr_cache = {}
    grid = sweep_grid(hi=s_max)
    per_L = {}
    for L in sizes:
        insts = [Instance.generate(L, wl.instance_seed("sa_batch", 100000 + 1000 * L + k), chain=k)
                 for k in range(n_inst)]
        reached = {t: [None] * n_inst for t in targets}
        batched_ms = {}
        eps_mean = {}
        for S in grid:
            jobs = [SAJob(inst, _thr(thr_cache, S, schedule), n_trials, seed) for inst in insts]
            b = Batch(jobs, graph=False)
            b.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            batched_ms[S] = (time.perf_counter() - t0) * 1e3
            b.close()
            m = np.array([float(epsilon(j.energy, inst.E_gs).mean()) for j, inst in zip(jobs, insts)])
            eps_mean[S] = float(m.mean())
            for t in targets:
                for k in range(n_inst):
                    if reached[t][k] is None and m[k] <= t:
                        reached[t][k] = S
            log(f"tteps L={L} S={S}: mean eps {m.mean():.4f}, batch {batched_ms[S]:.2f} ms, "
                f"reached {[sum(x is not None for x in reached[t]) for t in targets]}")
            if all(x is not None for x in reached[min(targets)]):
                break
        res_L = {"N": L ** 3, "eps_mean_by_S": eps_mean, "targets": {}}
        for t in targets:
            Ss = reached[t]
            if any(x is None for x in Ss):
                res_L["targets"][str(t)] = {"censored": True, "reached": int(sum(x is not None for x in Ss)),
                                            "S_max": grid[-1] if len(eps_mean) == len(grid) else max(eps_mean)}
                continue
            # plain: one trial, one launch (the kernels are warm from the
            # batched runs); timed on the first plain_inst instances
            plain = []
            for k, inst in enumerate(insts[:plain_inst]):
                thr = _thr(thr_cache, Ss[k], schedule)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sa_anneal(inst, thr, 1, seed)
                torch.cuda.synchronize()
                plain.append((time.perf_counter() - t0) * 1e3)
            batched = [batched_ms[S] / (n_inst * n_trials) for S in Ss]
            entry = {"censored": False, "S_star": Ss, "plain_ms": float(np.mean(plain)),
                     "plain_instances_timed": len(plain),
                     "batched_ms_per_trial": float(np.mean(batched))}
            if served:
                entry["served_ms"] = _served_latency(torch, insts, Ss, n_trials, seed, thr_cache, schedule)
            res_L["targets"][str(t)] = entry
        per_L[L] = res_L
    fits = {}
    for t in targets:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values()]
        pts = [(N, e) for N, e in pts if not e["censored"]]
        fits[str(t)] = {form: _fit([N for N, _ in pts], [e[key] for _, e in pts])
                        for form, key in (("plain", "plain_ms"), ("batched", "batched_ms_per_trial"),
                                          ("served", "served_ms")) if pts and key in pts[0][1]}
    return {"per_L": {str(L): v for L, v in per_L.items()}, "fits": fits,
            "n_inst": n_inst, "n_trials": n_trials, "grid": grid, "schedule": list(schedule)}


def _served_latency(torch, insts, Ss, n_trials, seed, thr_cache, schedule):
    from .serving import Server, SG_REQ_DONE
    srv = Server(max_active=8192, chunk_sweeps=512, large_slots=max(8, len(insts) * n_trials),
                 chunk_attempts=1 << 24)
    ids = []
    bufs = []
    for k, inst in enumerate(insts):
        thr = _thr(thr_cache, Ss[k], schedule)
        for r in range(n_trials):
            sp = torch.empty(inst.L ** 3, dtype=torch.int8, device="cuda")
            en = torch.empty(1, dtype=torch.int32, device="cuda")
            bufs.append((sp, en))
            ids.append(srv.submit(inst, thr, seed, r, sp, en))
    srv.wait(600.0)
    lat = [(s["t_done"] - s["t_arrival"]) * 1e3 for s in (srv.poll(i) for i in ids) if s["state"] == SG_REQ_DONE]
    srv.close()
    return float(np.mean(lat))


def _fit(N, T):
    """Least-squares fit of T = a N^alpha + b; returns a, alpha, b (None with
    fewer than three points)."""
    if len(N) < 3:
        return None
    from scipy.optimize import curve_fit
    N = np.asarray(N, np.float64)
    T = np.asarray(T, np.float64)

    def f(n, a, alpha, b):
        return a * np.power(n / N[0], alpha) + b
    try:
        p, _ = curve_fit(f, N, T, p0=(T[0], 1.0, 0.0), maxfev=20000)
    except Exception:
        return None
    return {"a_at_N0": float(p[0]), "alpha": float(p[1]), "b": float(p[2]), "N0": float(N[0])}
