"""Hyper-parameter tuning and the alpha(eps) experiment of App. D, on the
tile-planted stand-in instances, with the device kernels.

App. D tunes each heuristic once per target eps and then measures TT-eps
versus size:

SA       geometric beta schedule.  At L = 10, for each of 20 instances and
         every (beta_min, beta_max) of the grid beta_min = 0.3, 0.5, ..., 3.3
         and beta_max = 3, 4, ..., 27, the smallest number of sweeps at which
         the mean eps over 20 independent runs reaches the target; the
         combination that minimises it is recorded per instance, and the
         averages over the instances of the optimal beta_min and beta_max fix
         the schedule for that target.  TT-eps is then measured at
         L = 20, 30, 40, 50, 56.
PT       geometric ladder tuned at L = 4 over beta_min = 0.1, 0.3, ..., 2.7,
         beta_max = 3, 4, ..., 19, sweeps 1..20 and 2..4 temperatures,
         without cluster moves, minimising temperatures x sweeps; TT-eps of
         PT with isoenergetic cluster moves (two copies, moves at every
         temperature) at L = 6, 8, 10, 12.
TT-eps   per instance: the smallest sweep count whose mean eps over 20
         trials reaches the target, and the mean wall time of a trial at that
         count; averaged over 20 instances; fit TT = a N^alpha + b (N = L^3,
         the paper's a L^(3 alpha) + b).

Readings where the paper is silent (each also in the design notes):
  * the sweep counts searched: a geometric grid (four points per octave for
    the tuning, two for the scaling runs), not every integer;
  * ties between grid points at an instance's minimal sweep count: the
    centroid (mean beta_min, mean beta_max) of the tied combinations; for PT
    the number of temperatures is the most frequent among the tied (and,
    across instances, among the instances' optima), the smaller on a tie;
  * PT's eps after s sweeps: the lowest energy any walker reached by then
    (best so far), as the ground-state search returns it;
  * "walltime of a trial": one plain call of one replica (one run) at the
    found sweep count, launch to completion; the batched form divides one
    launch of all trials of all instances by their number.

The per-instance mean eps is computed from the exact energy sums of the
epsilon_stats kernel.  The functions without a GPU argument are pure and
tested on the host.
"""
from __future__ import annotations

import time
from collections import Counter

import numpy as np

from . import (Batch, Instance, SAJob, epsilon_stats, exchange_table_width, make_exchange_thresholds,
               make_schedule, make_thresholds, mean_epsilon, pt_run, pticm_run, sa_anneal, to_device_u32)
from . import workloads as wl

TARGETS = (0.03, 0.04, 0.05)


# ---------------------------------------------------------------------------
# grids and pure helpers (host, tested without a GPU)
# ---------------------------------------------------------------------------

def _steps(lo: float, hi: float, step: float) -> list:
    n = int(np.floor((hi - lo) / step + 1e-9)) + 1
    return [round(lo + k * step, 10) for k in range(n)]


def appd_sa_grid() -> tuple:
    """App. D's SA temperature ranges: beta_min 0.3 .. 3.3 by 0.2, beta_max
    3 .. 27 by 1 (400 combinations)."""
    return _steps(0.3, 3.3, 0.2), _steps(3.0, 27.0, 1.0)


def appd_pt_grid() -> tuple:
    """App. D's PT tuning grid: beta_min from 0.1 in steps of 0.2 up to
    2.8, beta_max 3 .. 19 by 1, sweeps 1 .. 20, temperatures 2 .. 4."""
    return _steps(0.1, 2.8, 0.2), _steps(3.0, 19.0, 1.0), list(range(1, 21)), [2, 3, 4]


def sweep_grid(lo: int = 16, hi: int = 32768, per_octave: int = 2) -> list:
    """Sweep counts round(lo 2^(k/per_octave)), distinct, up to hi."""
    out, k = [], 0
    while True:
        s = int(round(lo * 2 ** (k / per_octave)))
        if s > hi:
            return out
        if not out or s != out[-1]:
            out.append(s)
        k += 1


def first_reached(eps_by_step, targets) -> dict:
    """eps_by_step: list of (S, mean eps per item) in increasing S.  For each
    target, per item the first S whose mean eps is at or below it (None:
    censored, never reached)."""
    n = len(eps_by_step[0][1]) if eps_by_step else 0
    out = {t: [None] * n for t in targets}
    for S, m in eps_by_step:
        for t in targets:
            r = out[t]
            for i in range(n):
                if r[i] is None and m[i] <= t:
                    r[i] = S
    return out


def instance_optimum(reached, params) -> dict | None:
    """reached[j]: the sweeps combination j needed (None: censored); params[j]:
    its (beta_min, beta_max).  The least sweeps and the centroid of the
    combinations that need exactly that many; None when none reaches."""
    ok = [(s, j) for j, s in enumerate(reached) if s is not None]
    if not ok:
        return None
    best = min(s for s, _ in ok)
    tied = [j for s, j in ok if s == best]
    p = np.array([params[j] for j in tied], np.float64)
    return {"sweeps": best, "beta_min": float(p[:, 0].mean()), "beta_max": float(p[:, 1].mean()),
            "tied": len(tied)}


def average_optimum(opts) -> dict | None:
    """Mean over the instances (censored ones dropped) of their optimal
    beta_min and beta_max."""
    ok = [o for o in opts if o is not None]
    if not ok:
        return None
    return {"beta_min": float(np.mean([o["beta_min"] for o in ok])),
            "beta_max": float(np.mean([o["beta_max"] for o in ok])),
            "instances": len(ok), "censored": len(opts) - len(ok),
            "mean_sweeps": float(np.mean([o["sweeps"] for o in ok]))}


def pt_instance_optimum(costs) -> dict | None:
    """costs: list of (T, beta_min, beta_max, sweeps or None).  The least
    temperatures x sweeps; among the tied, the most frequent T (smaller on a
    tie) and the centroid of their betas."""
    ok = [(T * s, T, b0, b1, s) for T, b0, b1, s in costs if s is not None]
    if not ok:
        return None
    best = min(c for c, *_ in ok)
    tied = [x for x in ok if x[0] == best]
    cnt = Counter(x[1] for x in tied)
    T = min(cnt, key=lambda k: (-cnt[k], k))
    sel = [x for x in tied if x[1] == T]
    return {"T": T, "cost": best, "sweeps": sel[0][4], "beta_min": float(np.mean([x[2] for x in sel])),
            "beta_max": float(np.mean([x[3] for x in sel])), "tied": len(tied)}


def pt_average_optimum(opts) -> dict | None:
    ok = [o for o in opts if o is not None]
    if not ok:
        return None
    cnt = Counter(o["T"] for o in ok)
    T = min(cnt, key=lambda k: (-cnt[k], k))
    return {"T": T, "beta_min": float(np.mean([o["beta_min"] for o in ok])),
            "beta_max": float(np.mean([o["beta_max"] for o in ok])), "instances": len(ok),
            "censored": len(opts) - len(ok), "T_votes": {str(k): v for k, v in sorted(cnt.items())}}


def fit_alpha(N, T):
    """Least-squares fit of T = a (N/N0)^alpha + b (N0 = the smallest N);
    None with fewer than three points or when the fit fails."""
    if len(N) < 3:
        return None
    from scipy.optimize import curve_fit
    N = np.asarray(N, np.float64)
    T = np.asarray(T, np.float64)
    N0 = float(N.min())

    def f(n, a, alpha, b):
        return a * np.power(n / N0, alpha) + b
    try:
        p, _ = curve_fit(f, N, T, p0=(max(T.min(), 1e-9), 1.0, 0.0), maxfev=50000)
    except Exception:
        return None
    return {"a_at_N0": float(p[0]), "alpha": float(p[1]), "b": float(p[2]), "N0": N0}


# ---------------------------------------------------------------------------
# device drivers
# ---------------------------------------------------------------------------

def _instances(workload: str, L: int, n: int, base: int):
    specs = [wl.InstanceSpec(L, wl.instance_seed(workload, base + 1000 * L + k), k) for k in range(n)]
    return [Instance.generate(s.L, s.seed, s.chain) for s in specs]


def _geometric_thr(b0: float, b1: float, S: int):
    return make_thresholds(make_schedule(1, b0, b1, S))


def sa_tune(torch, L=10, n_inst=20, n_runs=20, targets=TARGETS, s_max=4096, per_octave=4, log=print):
    """App. D's SA range tuning at L: every (beta_min, beta_max) of the grid x
    every instance, n_runs runs each, one batched launch per sweep count."""
    bmins, bmaxs = appd_sa_grid()
    params = [(b0, b1) for b0 in bmins for b1 in bmaxs]
    seed = wl.philox_seed("sa_small") ^ 0xA9D
    insts = _instances("sa_small", L, n_inst, 70000)
    egs_all = [i.E_gs for i in insts]
    P, I = len(params), len(insts)
    reached = {t: np.full((P, I), -1, np.int64) for t in targets}
    grid = [s for s in sweep_grid(1, s_max, per_octave)]
    t0 = time.perf_counter()
    attempts = 0.0
    for S in grid:
        todo = [(p, i) for p in range(P) for i in range(I) if reached[min(targets)][p, i] < 0]
        if not todo:
            break
        ps = sorted({p for p, _ in todo})
        thr = {p: to_device_u32(_geometric_thr(params[p][0], params[p][1], S)) for p in ps}
        E = torch.empty((len(todo), n_runs), dtype=torch.int32, device="cuda")
        jobs = [SAJob(insts[i], thr[p], n_runs, seed, energy=E[k]) for k, (p, i) in enumerate(todo)]
        b = Batch(jobs, graph=False)
        b.launch()
        egs = torch.tensor([egs_all[i] for _, i in todo], dtype=torch.int64, device="cuda")
        st = epsilon_stats(E, egs)
        m = mean_epsilon(st, egs)
        b.close()
        attempts += len(todo) * n_runs * S * L ** 3
        for k, (p, i) in enumerate(todo):
            for t in targets:
                if reached[t][p, i] < 0 and m[k] <= t:
                    reached[t][p, i] = S
        log(f"sa tune L={L} S={S}: {len(todo)} pairs, reached {[int((reached[t] >= 0).sum()) for t in targets]}")
    out = {"L": L, "n_inst": I, "n_runs": n_runs, "grid": {"beta_min": bmins, "beta_max": bmaxs},
           "sweeps_searched": grid, "device_s": time.perf_counter() - t0, "attempts": attempts, "targets": {}}
    for t in targets:
        opts = [instance_optimum([int(reached[t][p, i]) if reached[t][p, i] >= 0 else None for p in range(P)],
                                 params) for i in range(I)]
        out["targets"][str(t)] = {"per_instance": opts, "schedule": average_optimum(opts)}
        log(f"sa tune target {t}: {out['targets'][str(t)]['schedule']}")
    return out


def sa_alpha(torch, schedules, sizes=(20, 30, 40, 50, 56), n_inst=20, n_trials=20, s_max=65536, log=print):
    """TT-eps of SA at each size for each target with its tuned geometric
    schedule (targets: {eps: (beta_min, beta_max)})."""
    seed = wl.philox_seed("serve") ^ 0x5A1
    per_L = {}
    for L in sizes:
        insts = _instances("sa_batch", L, n_inst, 500000)
        egs = torch.tensor([i.E_gs for i in insts], dtype=torch.int64, device="cuda")
        res_L = {"N": L ** 3, "targets": {}}
        for t, (b0, b1) in schedules.items():
            found = [None] * n_inst
            eps_by_S = []
            for S in sweep_grid(16, s_max, 2):
                E = torch.empty((n_inst, n_trials), dtype=torch.int32, device="cuda")
                thr = to_device_u32(_geometric_thr(b0, b1, S))
                jobs = [SAJob(inst, thr, n_trials, seed, energy=E[k]) for k, inst in enumerate(insts)]
                bt = Batch(jobs, graph=False)
                bt.launch()
                m = mean_epsilon(epsilon_stats(E, egs), egs)
                bt.close()
                eps_by_S.append((S, m))
                for k in range(n_inst):
                    if found[k] is None and m[k] <= t:
                        found[k] = S
                if all(f is not None for f in found):
                    break
            entry = {"S_star": found, "mean_eps_by_S": {str(S): float(m.mean()) for S, m in eps_by_S}}
            if any(f is None for f in found):
                entry["censored"] = True
                res_L["targets"][str(t)] = entry
                log(f"sa alpha L={L} eps={t}: censored ({sum(f is None for f in found)} instances)")
                continue
            # plain: every trial of every instance as its own call, launch to
            # completion (App. D: the mean over the 20 trials, then over the
            # instances)
            thr_of = {S: to_device_u32(_geometric_thr(b0, b1, S)) for S in set(found)}
            sa_anneal(insts[0], thr_of[found[0]], 1, seed)
            torch.cuda.synchronize()
            per_inst = []
            for k, inst in enumerate(insts):
                ms = []
                for r in range(n_trials):
                    t0 = time.perf_counter()
                    sa_anneal(inst, thr_of[found[k]], 1, seed, rep0=r)
                    torch.cuda.synchronize()
                    ms.append((time.perf_counter() - t0) * 1e3)
                per_inst.append(float(np.mean(ms)))
            # batched: all trials of all instances, each at its own count, in
            # one launch, divided by the number of trials
            E = torch.empty((n_inst, n_trials), dtype=torch.int32, device="cuda")
            jobs = [SAJob(inst, thr_of[found[k]], n_trials, seed, energy=E[k]) for k, inst in enumerate(insts)]
            bt = Batch(jobs, graph=True)
            bt.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bt.launch()
            torch.cuda.synchronize()
            batched = (time.perf_counter() - t0) * 1e3 / (n_inst * n_trials)
            bt.close()
            entry.update({"censored": False, "plain_ms": float(np.mean(per_inst)), "plain_ms_per_instance": per_inst,
                          "batched_ms_per_trial": batched, "S_star_mean": float(np.mean(found))})
            res_L["targets"][str(t)] = entry
            log(f"sa alpha L={L} eps={t}: S* mean {np.mean(found):.0f}, plain {np.mean(per_inst):.3f} ms, "
                f"batched {batched:.4f} ms/trial")
        per_L[L] = res_L
    fits = {}
    for t in schedules:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values() if not v["targets"][str(t)]["censored"]]
        fits[str(t)] = {form: fit_alpha([N for N, _ in pts], [e[key] for _, e in pts])
                        for form, key in (("plain", "plain_ms"), ("batched", "batched_ms_per_trial"))}
    return {"sizes": list(sizes), "per_L": {str(L): v for L, v in per_L.items()}, "fits": fits,
            "schedules": {str(t): list(v) for t, v in schedules.items()}}


def _pt_tables(T, b0, b1):
    beta = make_schedule(1, b0, b1, T)
    M = exchange_table_width(beta)
    return to_device_u32(make_thresholds(beta)), to_device_u32(make_exchange_thresholds(beta, M))


def _best_so_far_eps(torch, trace, E_gs):
    """Mean eps over the runs of the lowest energy reached by each step
    (trace: device int32 [runs][steps] of per-step minima)."""
    best = torch.cummin(trace, dim=1).values.t().contiguous()
    return mean_epsilon(epsilon_stats(best, [E_gs] * best.shape[0]), E_gs)


def pt_tune(torch, L=4, n_inst=20, n_runs=20, targets=TARGETS, log=print):
    """App. D's PT ladder tuning at L (no cluster moves): every (T, beta_min,
    beta_max) x instance, one run of 20 steps per call gives every sweep
    count 1..20 (a run's first s steps do not depend on its length)."""
    bmins, bmaxs, sweeps, Ts = appd_pt_grid()
    seed = wl.philox_seed("pt") ^ 0xA9D
    insts = _instances("pt", L, n_inst, 70000)
    S = max(sweeps)
    costs = {t: [[] for _ in insts] for t in targets}
    t0 = time.perf_counter()
    for T in Ts:
        for b0 in bmins:
            for b1 in bmaxs:
                thr, thrx = _pt_tables(T, b0, b1)
                for k, inst in enumerate(insts):
                    out = pt_run(inst, thr, thrx, n_runs, S, seed, want_trace=True)
                    m = _best_so_far_eps(torch, out["emin_trace"], inst.E_gs)
                    for t in targets:
                        hit = np.nonzero(m <= t)[0]
                        costs[t][k].append((T, b0, b1, int(hit[0]) + 1 if len(hit) else None))
        log(f"pt tune L={L} T={T} done")
    out = {"L": L, "n_inst": n_inst, "n_runs": n_runs,
           "grid": {"beta_min": bmins, "beta_max": bmaxs, "sweeps": sweeps, "temperatures": Ts},
           "device_s": time.perf_counter() - t0, "targets": {}}
    for t in targets:
        opts = [pt_instance_optimum(c) for c in costs[t]]
        out["targets"][str(t)] = {"per_instance": opts, "ladder": pt_average_optimum(opts)}
        log(f"pt tune target {t}: {out['targets'][str(t)]['ladder']}")
    return out


def pticm_alpha(torch, ladders, sizes=(6, 8, 10, 12), n_inst=20, n_trials=20, n_steps=4000, log=print):
    """TT-eps of PT with isoenergetic cluster moves (two copies, moves at every
    temperature) at each size for each target with its tuned ladder
    (ladders: {eps: (T, beta_min, beta_max)})."""
    seed = wl.philox_seed("pt") ^ 0x1C3
    per_L = {}
    for L in sizes:
        insts = _instances("pt", L, n_inst, 600000)
        res_L = {"N": L ** 3, "targets": {}}
        for t, (T, b0, b1) in ladders.items():
            thr, thrx = _pt_tables(T, b0, b1)
            found, batch_ms = [], []
            for inst in insts:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = pticm_run(inst, thr, thrx, n_trials, n_steps, seed, icm_from=0, want_trace=True)
                torch.cuda.synchronize()
                batch_ms.append((time.perf_counter() - t0) * 1e3)
                m = _best_so_far_eps(torch, out["emin_trace"], inst.E_gs)
                hit = np.nonzero(m <= t)[0]
                found.append(int(hit[0]) + 1 if len(hit) else None)
            entry = {"steps_star": found}
            if any(f is None for f in found):
                entry["censored"] = True
                res_L["targets"][str(t)] = entry
                continue
            pticm_run(insts[0], thr, thrx, 1, found[0], seed, icm_from=0)
            torch.cuda.synchronize()
            per_inst = []
            for k, inst in enumerate(insts):
                ms = []
                for r in range(n_trials):
                    t0 = time.perf_counter()
                    pticm_run(inst, thr, thrx, 1, found[k], seed, run0=r, icm_from=0)
                    torch.cuda.synchronize()
                    ms.append((time.perf_counter() - t0) * 1e3)
                per_inst.append(float(np.mean(ms)))
            # batched: the n_trials-run launch's time per step and run, at
            # each instance's step count
            ms_step_run = float(np.mean(batch_ms)) / n_steps / n_trials
            entry.update({"censored": False, "steps_star_mean": float(np.mean(found)),
                          "plain_ms": float(np.mean(per_inst)), "plain_ms_per_instance": per_inst,
                          "batched_ms": float(np.mean(found)) * ms_step_run})
            res_L["targets"][str(t)] = entry
            log(f"pticm alpha L={L} eps={t}: steps* mean {np.mean(found):.1f}, plain {np.mean(per_inst):.3f} ms")
        per_L[L] = res_L
    fits = {}
    for t in ladders:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values() if not v["targets"][str(t)]["censored"]]
        fits[str(t)] = {form: fit_alpha([N for N, _ in pts], [e[key] for _, e in pts])
                        for form, key in (("plain", "plain_ms"), ("batched", "batched_ms"))}
    return {"sizes": list(sizes), "per_L": {str(L): v for L, v in per_L.items()}, "fits": fits,
            "ladders": {str(t): list(v) for t, v in ladders.items()}}


def alpha_table(res) -> list:
    """Rows (eps, SA alpha plain/batched, PT+ICM alpha plain/batched)."""
    rows = []
    for t in TARGETS:
        row = {"eps": t}
        for name in ("sa_alpha", "pticm_alpha"):
            f = res.get(name, {}).get("fits", {}).get(str(t), {})
            for form in ("plain", "batched"):
                v = f.get(form)
                row[f"{name}_{form}"] = None if v is None else v["alpha"]
        rows.append(row)
    return rows


def run(torch, log=print, sa_sizes=(20, 30, 40, 50, 56), pt_sizes=(6, 8, 10, 12)):
    """The whole App. D form: SA tuning at L = 10 and PT tuning at L = 4, then
    TT-eps and alpha(eps) of SA and of PT with cluster moves."""
    out = {"sa_tune": sa_tune(torch, log=log), "pt_tune": pt_tune(torch, log=log)}
    sched = {t: (v["schedule"]["beta_min"], v["schedule"]["beta_max"])
             for t, v in ((float(k), v) for k, v in out["sa_tune"]["targets"].items()) if v["schedule"]}
    out["sa_alpha"] = sa_alpha(torch, sched, sizes=sa_sizes, log=log)
    ladders = {t: (v["ladder"]["T"], v["ladder"]["beta_min"], v["ladder"]["beta_max"])
               for t, v in ((float(k), v) for k, v in out["pt_tune"]["targets"].items()) if v["ladder"]}
    out["pticm_alpha"] = pticm_alpha(torch, ladders, sizes=pt_sizes, log=log)
    out["alpha_table"] = alpha_table(out)
    for r in out["alpha_table"]:
        log(f"alpha(eps={r['eps']}): {r}")
    return out


# ---------------------------------------------------------------------------
# PT TT-eps with a fixed ladder, one run alone vs spread over work groups
# ---------------------------------------------------------------------------

def pt_tteps(torch, T=8, beta_max=2.0, sizes=(6, 8, 10, 12), n_inst=20, n_runs=20,
             targets=TARGETS, n_steps=4000, log=print):
    """PT TT-eps versus N with the ladder (T, geometric 0.2 -> beta_max): the
    time per step of one run alone (pt_run), of one run spread over work
    groups (sg_pt_run_split) and of n_runs runs per launch."""
    seed = wl.philox_seed("pt") ^ 0x71
    thr, thrx = _pt_tables(T, 0.2, beta_max)
    per_L = {}
    for L in sizes:
        insts = _instances("pt", L, n_inst, 0)
        times = {}
        for form, groups in (("plain", 1), ("split", 0)):
            pt_run(insts[0], thr, thrx, 1, 50, seed, groups=groups)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pt_run(insts[0], thr, thrx, 1, n_steps, seed, groups=groups)
            torch.cuda.synchronize()
            times[form] = (time.perf_counter() - t0) * 1e3 / n_steps
        steps = {t: [] for t in targets}
        batch_ms = []
        for inst in insts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = pt_run(inst, thr, thrx, n_runs, n_steps, seed, want_trace=True)
            torch.cuda.synchronize()
            batch_ms.append((time.perf_counter() - t0) * 1e3)
            m = _best_so_far_eps(torch, out["emin_trace"], inst.E_gs)
            for t in targets:
                hit = np.nonzero(m <= t)[0]
                steps[t].append(int(hit[0]) + 1 if len(hit) else None)
        times["batched"] = float(np.mean(batch_ms)) / n_steps / n_runs
        entry = {"N": L ** 3, "ms_per_step": times, "targets": {}}
        for t in targets:
            st = steps[t]
            if any(x is None for x in st):
                entry["targets"][str(t)] = {"censored": True}
                continue
            entry["targets"][str(t)] = {"censored": False, "steps_mean": float(np.mean(st)),
                                        **{f"{f}_ms": float(np.mean(st)) * v for f, v in times.items()}}
        log(f"pt tteps L={L}: {entry}")
        per_L[L] = entry
    fits = {}
    for t in targets:
        pts = [(v["N"], v["targets"][str(t)]) for v in per_L.values() if not v["targets"][str(t)]["censored"]]
        fits[str(t)] = {f: fit_alpha([N for N, _ in pts], [e[f"{f}_ms"] for _, e in pts])
                        for f in ("plain", "split", "batched")}
    return {"T": T, "beta_max": beta_max, "per_L": {str(L): v for L, v in per_L.items()}, "fits": fits}
