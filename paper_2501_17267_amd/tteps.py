"""Time-to-epsilon (TT-eps) versus system size, in the form of App. D.

For each lattice size L: n_inst instances, n_trials independent annealing
runs (one read each) per instance; the sweep count S walks a grid of powers
of sqrt(2); an instance reaches a target eps at the smallest S whose mean eps
over its trials is at or below the target (Eq. 2; App. D's criterion, from
the exact energy sums of the epsilon_stats kernel).  Its TT-eps is the time
of one trial at that S, measured three ways:

  plain    every trial of every instance as its own sa_anneal call of one
           replica, launch to completion; the mean over the trials, then over
           the instances (App. D's walltime average)
  batched  all trials of all instances of the size, each instance at its
           own S, in one batched launch, divided by the number of trials
  served   the same trials submitted together to the anneal server: the
           time to serve them all divided by their number (a per-trial cost,
           comparable with the batched form), and, apart, the mean latency
           of a request in that burst (which includes its queueing)

The results at one S are identical across the three forms (same counters),
so they compare at equal eps.  TT-eps(L) is the mean over instances; a fit
TT-eps = a N^alpha + b (N = L^3, App. D) gives the scaling exponent alpha.
Sizes whose instances do not all reach a target by S_max are reported as
censored for that target.
"""
from __future__ import annotations

import time

import numpy as np

from . import Batch, Instance, SAJob, epsilon_stats, make_schedule, make_thresholds, mean_epsilon, sa_anneal, \
    to_device_u32
from . import workloads as wl
from .tuning import first_reached, fit_alpha, sweep_grid

# the two names the earlier harness exported
_fit = fit_alpha


def _thr(cache, S, schedule=(0, 0.1, 3.0)):
    key = (S,) + tuple(schedule)
    if key not in cache:
        kind, b0, b1 = schedule
        cache[key] = to_device_u32(make_thresholds(make_schedule(kind, b0, b1, S)))
    return cache[key]


def run(torch, sizes=(8, 12, 16, 20, 24, 32, 64), n_inst=20, n_trials=20, targets=(0.01, 0.03, 0.04, 0.05),
        s_max=32768, log=print, served=True, schedule=(0, 0.1, 3.0)):
    """schedule: (kind, beta0, beta1) of every anneal (0 linear, 1 geometric)."""
    seed = wl.philox_seed("serve") ^ 0x77
    thr_cache = {}
    grid = sweep_grid(hi=s_max)
    per_L = {}
    for L in sizes:
        insts = [Instance.generate(L, wl.instance_seed("sa_batch", 100000 + 1000 * L + k), chain=k)
                 for k in range(n_inst)]
        egs = torch.tensor([i.E_gs for i in insts], dtype=torch.int64, device="cuda")
        eps_by_S = []
        for S in grid:
            E = torch.empty((n_inst, n_trials), dtype=torch.int32, device="cuda")
            jobs = [SAJob(inst, _thr(thr_cache, S, schedule), n_trials, seed, energy=E[k])
                    for k, inst in enumerate(insts)]
            b = Batch(jobs, graph=False)
            b.launch()
            m = mean_epsilon(epsilon_stats(E, egs), egs)
            b.close()
            eps_by_S.append((S, m))
            reached = first_reached(eps_by_S, targets)
            log(f"tteps L={L} S={S}: mean eps {m.mean():.4f}, reached "
                f"{[sum(x is not None for x in reached[t]) for t in targets]}")
            if all(x is not None for x in reached[min(targets)]):
                break
        reached = first_reached(eps_by_S, targets)
        res_L = {"N": L ** 3, "eps_mean_by_S": {str(S): float(m.mean()) for S, m in eps_by_S}, "targets": {}}
        for t in targets:
            Ss = reached[t]
            if any(x is None for x in Ss):
                res_L["targets"][str(t)] = {"censored": True, "reached": int(sum(x is not None for x in Ss)),
                                            "S_max": eps_by_S[-1][0]}
                continue
            entry = {"censored": False, "S_star": Ss}
            entry.update(_timings(torch, insts, Ss, n_trials, seed, thr_cache, schedule, served))
            res_L["targets"][str(t)] = entry
            log(f"tteps L={L} eps={t}: {entry}")
        per_L[L] = res_L
    fits = {}
    for t in targets:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values()]
        pts = [(N, e) for N, e in pts if not e["censored"]]
        forms = (("plain", "plain_ms"), ("batched", "batched_ms_per_trial"), ("served", "served_ms_per_trial"))
        fits[str(t)] = {form: fit_alpha([N for N, _ in pts], [e[key] for _, e in pts])
                        for form, key in forms if pts and key in pts[0][1]}
    return {"per_L": {str(L): v for L, v in per_L.items()}, "fits": fits,
            "n_inst": n_inst, "n_trials": n_trials, "grid": grid, "schedule": list(schedule)}


def _timings(torch, insts, Ss, n_trials, seed, thr_cache, schedule, served):
    """Plain, batched and served time of one trial at each instance's S*."""
    sa_anneal(insts[0], _thr(thr_cache, Ss[0], schedule), 1, seed)
    torch.cuda.synchronize()
    per_inst = []
    for k, inst in enumerate(insts):
        thr = _thr(thr_cache, Ss[k], schedule)
        ms = []
        for r in range(n_trials):
            t0 = time.perf_counter()
            sa_anneal(inst, thr, 1, seed, rep0=r)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        per_inst.append(float(np.mean(ms)))
    E = torch.empty((len(insts), n_trials), dtype=torch.int32, device="cuda")
    jobs = [SAJob(inst, _thr(thr_cache, Ss[k], schedule), n_trials, seed, energy=E[k])
            for k, inst in enumerate(insts)]
    b = Batch(jobs, graph=True)
    b.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.launch()
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) * 1e3 / (len(insts) * n_trials)
    b.close()
    out = {"plain_ms": float(np.mean(per_inst)), "plain_ms_per_instance": per_inst,
           "batched_ms_per_trial": batched}
    if served:
        out.update(_served(torch, insts, Ss, n_trials, seed, thr_cache, schedule))
    return out


def _served(torch, insts, Ss, n_trials, seed, thr_cache, schedule):
    from .serving import Server, SG_REQ_DONE
    srv = Server(max_active=8192, chunk_sweeps=512, large_slots=max(8, len(insts) * n_trials),
                 chunk_attempts=1 << 24)
    ids = []
    bufs = []
    t0 = srv.now()
    for k, inst in enumerate(insts):
        thr = _thr(thr_cache, Ss[k], schedule)
        for r in range(n_trials):
            sp = torch.empty(inst.L ** 3, dtype=torch.int8, device="cuda")
            en = torch.empty(1, dtype=torch.int32, device="cuda")
            bufs.append((sp, en))
            ids.append(srv.submit(inst, thr, seed, r, sp, en))
    srv.wait(600.0)
    st = [srv.poll(i) for i in ids]
    srv.close()
    done = [s for s in st if s["state"] == SG_REQ_DONE]
    span = max(s["t_done"] for s in done) - t0
    lat = [(s["t_done"] - s["t_arrival"]) * 1e3 for s in done]
    return {"served_ms_per_trial": span * 1e3 / len(done), "served_mean_latency_ms_in_burst": float(np.mean(lat))}
