"""Hyper-parameter tuning and the alpha(eps) experiment of App. D.

The paper tunes SA's inverse-temperature range at one small size and the PT
ladder at another, then measures TT-eps versus N at eps = 3, 4 and 5 % and
fits a N^alpha + b at each eps (alpha(eps)).  Here, on the tile-planted
stand-in instances, with the device kernels:

sa_beta_grid   SA schedules (kind, beta0, beta1) at L = 10: for each, the
               smallest sweep count of the sqrt(2) grid at which the mean eps
               over 20 trials reaches the target, per instance (batched
               launches of 20 instances x 20 trials); the schedule with the
               smallest mean count wins.
pt_ladder_grid PT ladders (T walkers, geometric 0.2 -> beta_max) at L = 6:
               the steps at which the mean over 20 runs of the best energy
               seen so far reaches the target, per instance; the ladder with
               the least work (steps x T sweeps) wins.
pt_tteps       PT (and PT with isoenergetic cluster moves) TT-eps versus N
               (L = 6, 8, 10, 12) at eps = 3, 4, 5 % with the chosen ladder:
               per instance one launch of 20 runs with the per-step
               minimum-energy trace; TT-eps = the time of the steps
               needed, from the measured time per step of one run alone
               (plain), of one run alone spread over work groups (split,
               PT only) and of the 20-run launch divided by 20 (batched).
"""
from __future__ import annotations

import time

import numpy as np

from . import (Batch, Instance, SAJob, epsilon, exchange_table_width, make_exchange_thresholds, make_schedule,
               make_thresholds, pt_run, pticm_run, to_device_u32)
from . import workloads as wl
from .tteps import _fit, sweep_grid


def sa_beta_grid(torch, L=10, n_inst=20, n_trials=20, target=0.03, s_max=8192,
                 kinds=(0, 1), beta0s=(0.05, 0.1, 0.3), beta1s=(1.5, 2.0, 3.0, 5.0), log=print):
    seed = wl.philox_seed("sa_small") ^ 0x5A
    specs = [wl.InstanceSpec(L, wl.instance_seed("sa_small", 7000 + k), k) for k in range(n_inst)]
    insts = [Instance.generate(s.L, s.seed, s.chain) for s in specs]
    grid = sweep_grid(hi=s_max)
    rows = []
    for kind in kinds:
        for b0 in beta0s:
            for b1 in beta1s:
                reached = [None] * n_inst
                for S in grid:
                    thr = to_device_u32(make_thresholds(make_schedule(kind, b0, b1, S)))
                    jobs = [SAJob(inst, thr, n_trials, seed) for inst in insts]
                    b = Batch(jobs, graph=False)
                    b.launch()
                    torch.cuda.synchronize()
                    b.close()
                    for k, (j, inst) in enumerate(zip(jobs, insts)):
                        if reached[k] is None and float(epsilon(j.energy, inst.E_gs).mean()) <= target:
                            reached[k] = S
                    if all(x is not None for x in reached):
                        break
                ok = all(x is not None for x in reached)
                row = {"kind": kind, "beta0": b0, "beta1": b1, "censored": not ok,
                       "mean_sweeps": float(np.mean(reached)) if ok else None,
                       "reached": int(sum(x is not None for x in reached))}
                log(f"sa grid {row}")
                rows.append(row)
    done = [r for r in rows if not r["censored"]]
    best = min(done, key=lambda r: r["mean_sweeps"]) if done else None
    return {"L": L, "target": target, "rows": rows, "best": best}


def _pt_tables(T, beta_max):
    beta = make_schedule(1, 0.2, beta_max, T)
    M = exchange_table_width(beta)
    return to_device_u32(make_thresholds(beta)), to_device_u32(make_exchange_thresholds(beta, M))


def _pt_call(inst, thr, thrx, n_runs, n_steps, seed, icm_from=None, want_trace=False, groups=1):
    """PT (icm_from None; groups as in pt_run) or PT with cluster moves from
    slot icm_from."""
    if icm_from is None:
        return pt_run(inst, thr, thrx, n_runs, n_steps, seed, want_trace=want_trace, groups=groups)
    return pticm_run(inst, thr, thrx, n_runs, n_steps, seed, icm_from=icm_from, want_trace=want_trace)


def _pt_steps_to_targets(torch, inst, thr, thrx, n_runs, n_steps, seed, targets, icm_from=None):
    """Run n_runs runs of n_steps; return ({target: steps or None}, ms of the call)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = _pt_call(inst, thr, thrx, n_runs, n_steps, seed, icm_from, want_trace=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    tr = out["emin_trace"].cpu().numpy().astype(np.int64)
    best = np.minimum.accumulate(tr, axis=1)                # best energy seen so far, per run
    eps_mean = ((best - inst.E_gs) / abs(inst.E_gs)).mean(axis=0)
    res = {}
    for t in targets:
        hit = np.nonzero(eps_mean <= t)[0]
        res[t] = int(hit[0]) + 1 if len(hit) else None
    return res, ms


def pt_ladder_grid(torch, L=6, n_inst=20, n_runs=20, target=0.03, n_steps=2000,
                   Ts=(8, 16, 32), beta_maxs=(2.0, 3.0, 5.0), icm=False, log=print):
    """With icm, each ladder is tried with cluster moves on every slot and on
    the colder half (icm_from = 0, T/2); the work counts both copies."""
    seed = wl.philox_seed("pt") ^ 0x3C
    specs = [wl.InstanceSpec(L, wl.instance_seed("pt", 100 + k), k) for k in range(n_inst)]
    insts = [Instance.generate(s.L, s.seed, s.chain) for s in specs]
    rows = []
    for T in Ts:
        for bm in beta_maxs:
            thr, thrx = _pt_tables(T, bm)
            for icm_from in ((0, T // 2) if icm else (None,)):
                steps = []
                for inst in insts:
                    r, _ = _pt_steps_to_targets(torch, inst, thr, thrx, n_runs, n_steps, seed, (target,), icm_from)
                    steps.append(r[target])
                ok = all(x is not None for x in steps)
                walkers = T * (2 if icm else 1)
                row = {"T": T, "beta_max": bm, "icm_from": icm_from, "censored": not ok,
                       "mean_steps": float(np.mean(steps)) if ok else None,
                       "mean_sweeps": float(np.mean(steps)) * walkers if ok else None,
                       "reached": int(sum(x is not None for x in steps))}
                log(f"pt{'+icm' if icm else ''} grid {row}")
                rows.append(row)
    done = [r for r in rows if not r["censored"]]
    best = min(done, key=lambda r: r["mean_sweeps"]) if done else None
    return {"L": L, "target": target, "rows": rows, "best": best}


def pt_tteps(torch, T=32, beta_max=3.0, sizes=(6, 8, 10, 12), n_inst=20, n_runs=20,
             targets=(0.03, 0.04, 0.05), n_steps=4000, icm_from=None, log=print):
    """icm_from None: PT; else PT with cluster moves from that slot."""
    seed = wl.philox_seed("pt") ^ 0x71
    thr, thrx = _pt_tables(T, beta_max)
    per_L = {}
    for L in sizes:
        specs = [wl.InstanceSpec(L, wl.instance_seed("pt", 1000 * L + k), k) for k in range(n_inst)]
        insts = [Instance.generate(s.L, s.seed, s.chain) for s in specs]
        # time per step of one run alone and of the n_runs launch
        _pt_call(insts[0], thr, thrx, 1, 50, seed, icm_from)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _pt_call(insts[0], thr, thrx, 1, n_steps, seed, icm_from)
        torch.cuda.synchronize()
        ms_step_plain = (time.perf_counter() - t0) * 1e3 / n_steps
        ms_step_split = None
        if icm_from is None:
            # the same run alone, spread over work groups (sg_pt_run_split)
            _pt_call(insts[0], thr, thrx, 1, 50, seed, groups=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _pt_call(insts[0], thr, thrx, 1, n_steps, seed, groups=0)
            torch.cuda.synchronize()
            ms_step_split = (time.perf_counter() - t0) * 1e3 / n_steps
        steps = {t: [] for t in targets}
        batch_ms = []
        for inst in insts:
            r, ms = _pt_steps_to_targets(torch, inst, thr, thrx, n_runs, n_steps, seed, targets, icm_from)
            batch_ms.append(ms)
            for t in targets:
                steps[t].append(r[t])
        ms_step_batched = float(np.mean(batch_ms)) / n_steps / n_runs
        entry = {"N": L ** 3, "ms_per_step_plain": ms_step_plain, "ms_per_step_batched": ms_step_batched,
                 "targets": {}}
        if ms_step_split is not None:
            entry["ms_per_step_split"] = ms_step_split
        for t in targets:
            st = steps[t]
            if any(x is None for x in st):
                entry["targets"][str(t)] = {"censored": True, "reached": int(sum(x is not None for x in st))}
                continue
            entry["targets"][str(t)] = {"censored": False, "steps_mean": float(np.mean(st)),
                                        "plain_ms": float(np.mean(st)) * ms_step_plain,
                                        "batched_ms": float(np.mean(st)) * ms_step_batched}
            if ms_step_split is not None:
                entry["targets"][str(t)]["split_ms"] = float(np.mean(st)) * ms_step_split
        log(f"pt{'' if icm_from is None else '+icm'} tteps L={L}: {entry}")
        per_L[L] = entry
    fits = {}
    for t in targets:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values() if not v["targets"][str(t)]["censored"]]
        forms = (("plain", "plain_ms"), ("batched", "batched_ms")) + ((("split", "split_ms"),)
                                                                    if icm_from is None else ())
        fits[str(t)] = {form: _fit([N for N, _ in pts], [e[key] for _, e in pts]) for form, key in forms}
    return {"T": T, "beta_max": beta_max, "icm_from": icm_from, "per_L": {str(L): v for L, v in per_L.items()},
            "fits": fits}


def run(torch, log=print):
    """The whole App. D form: tune SA and PT, then alpha(eps) for both."""
    from . import tteps as tt
    sa = sa_beta_grid(torch, log=log)
    pt = pt_ladder_grid(torch, log=log)
    out = {"sa_grid": sa, "pt_grid": pt}
    if sa["best"]:
        b = sa["best"]
        out["sa_alpha"] = tt.run(torch, sizes=(8, 12, 16, 20, 24, 32), targets=(0.03, 0.04, 0.05),
                                 served=False, log=log, schedule=(b["kind"], b["beta0"], b["beta1"]))
    if pt["best"]:
        out["pt_alpha"] = pt_tteps(torch, T=pt["best"]["T"], beta_max=pt["best"]["beta_max"], log=log)
    icm = pt_ladder_grid(torch, Ts=(4, 8, 16), beta_maxs=(2.0, 3.0), icm=True, log=log)
    out["pticm_grid"] = icm
    if icm["best"]:
        b = icm["best"]
        out["pticm_alpha"] = pt_tteps(torch, T=b["T"], beta_max=b["beta_max"], icm_from=b["icm_from"], log=log)
    return out
