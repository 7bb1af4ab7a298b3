#!/usr/bin/env python3
"""Throughput benchmark of the annealing hot path on one MI355X.

A step is one pass of the whole path over the uneven batch: 4096 synthetic
tile-planted instances with L drawn from {6, 8, 10, 12, 16, 20}, 64 replicas
each, sweep budgets drawn from {128, 256, 512, 1024}, beta linear 0.1 -> 3.0
(initial spins from the init stream, checkerboard Metropolis sweeps, final
energies), launched as one captured hipGraph of per-size kernels, followed by
the per-instance optimality-gap statistics (Eq. 2; epsilon_stats).
Instances, schedules and tables are materialised before the timed region
(their host cost is reported apart).

Prints ONE JSON line: metric, value (spin-flip attempts/s), the batched form
against plain per-instance calls on a stratified subset (bit-identical, so at
equal eps), roofline of the dominant launch, the oracle timed on the host
cores (cpu_baseline), and the 48-instance batched workload (L = 8/12/16,
1024 replicas, 256 sweeps) under "sa_batch".

  python bench.py [--steps K] [--warmup W] [--workload uneven|sa_batch|...]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts (CDNA4)
N_CU = 256
CLOCK_HZ = 2.4e9
LANES_PER_CU = 64                      # 4 SIMD x 16 lanes, one 32-bit op each per clock
VALU32_PEAK = N_CU * LANES_PER_CU * CLOCK_HZ   # 39.3 T 32-bit lane-ops/s
HBM_PEAK_GBS = 8000.0

# Algorithmic work per spin-flip attempt in 32-bit VALU issue slots (one
# slot = one instruction on one lane; on gfx950 the 32x32->64 multiply-add
# and the 3-input xor issue at full rate, measured with --workload microbench):
#   Philox4x32-10 shared by 4 proposals: 10 rounds x (2 products + 2 xor3) / 4 = 10
#   local field h = sum of 6 couplings x neighbour spins: 6 multiply-adds      = 6
#   acceptance: k = -s h, k <= 0 test, u < thr[k] compare, flip select          = 4
OPS_PER_ATTEMPT = 20

KERNEL_SOURCES = ["device.hpp", "sweep.hpp", "sa_kernel.hpp", "sa_launch.hpp", "sa.hip", "batch.hip"]
TRAFFIC_SUMMARY = {"sa_batch": os.path.join(ROOT, "profiles", "k_sa_sa_batch_hbm_traffic.md"),
                   "uneven": os.path.join(ROOT, "profiles", "k_sa_uneven_hbm_traffic.md")}
COUNTER_SUMMARY = {"sa_batch": os.path.join(ROOT, "profiles", "k_sa_sa_batch_sq_counters.md"),
                   "uneven": os.path.join(ROOT, "profiles", "k_sa_uneven_sq_counters.md")}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_17267_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summary_json(path):
    """The json block of a committed rocprofv3 summary, or None when it is
    missing or the kernel sources changed since it was taken."""
    import re
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d


def measured_traffic(workload="uneven"):
    """HBM bytes per batched launch from the committed FETCH_SIZE/WRITE_SIZE
    summary of that workload (None when stale or absent)."""
    return _summary_json(TRAFFIC_SUMMARY[workload])


def measured_valu(workload="uneven"):
    """Counted VALU lane-slots per attempt from the committed SQ counter
    summary of that workload (None when stale or absent)."""
    return _summary_json(COUNTER_SUMMARY[workload])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uneven", choices=["sa_batch", "sa_small", "plain", "pt", "uneven", "serve", "tteps", "fragment", "fragment_call", "tn", "tuning", "pt_tteps", "wide", "pticm", "large", "tn_call", "microbench",
                             "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pt-groups", type=int, default=0,
                    help="pt: work groups per run (0: as many as fill the device, 1: pt_run)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work of the oracle sample")
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--variants", default=None,
                    help="fixed launch shapes instead of autotuning, e.g. 8=2,12=3,16=3 "
                         "(to profile exactly the shapes an earlier run selected)")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: measured seconds")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: requests per second")
    ap.add_argument("--chunk", type=int, default=512, help="serve: most sweeps per chunk")
    ap.add_argument("--chunk-attempts", type=int, default=1 << 24,
                    help="serve: target spin-flip attempts per request per chunk")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="hardware queues for this process (GPU_MAX_HW_QUEUES, <= 32); "
                         "serve defaults to 16, one per lattice-size stream")
    ap.add_argument("--no-graph-compare", action="store_true",
                    help="sa_batch: skip timing the same schedule replayed as a hipGraph")
    ap.add_argument("--no-extra", action="store_true",
                    help="uneven: skip the sa_batch and plain-call legs (for profiling the launch)")
    ap.add_argument("--plain-stride", type=int, default=32,
                    help="uneven: plain per-instance calls on every n-th job")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def build_sa_batch(sg, wl, torch, graph=False):
    w = wl.sa_batch()
    t0 = time.perf_counter()
    beta = sg.make_schedule(w.kind, w.beta0, w.beta1, w.n_sweeps)
    thr_h = sg.make_thresholds(beta, sg.SG_K_MAX)
    thr = sg.to_device_u32(thr_h)
    insts = [sg.Instance.generate(s.L, s.seed, s.chain) for s in w.instances]
    t_host = time.perf_counter() - t0
    E_all = torch.empty((len(insts), w.n_rep), dtype=torch.int32, device="cuda")
    jobs = [sg.SAJob(inst, thr, w.n_rep, w.seed, energy=E_all[k]) for k, inst in enumerate(insts)]
    batch = sg.Batch(jobs, graph=graph)
    return w, insts, jobs, batch, thr_h, t_host, E_all


def run_eps(sg, E_all, egs, out, stream):
    """Per-instance gap statistics of the batch (one epsilon_stats launch)."""
    out["st"] = sg.epsilon_stats(E_all, egs, targets=(0.01, 0.03, 0.05), stream=stream)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, unchanged, on a bounded sample of the workload
# ---------------------------------------------------------------------------

def cpu_baseline_sa(w, thr_h, target_s):
    import concurrent.futures as cf

    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    specs = {}
    for s in w.instances:
        specs.setdefault(s.L, s)
    inst = {L: oracle.make_instance(L, s.cls, s.seed) for L, s in specs.items()}
    # calibrate on one replica of the smallest lattice
    Ls = sorted(specs)
    t0 = time.perf_counter()
    oracle.sa_run(Ls[0], inst[Ls[0]][0], w.seed, specs[Ls[0]].chain, thr_h, n_rep=1, rep0=0)
    per_att = (time.perf_counter() - t0) / (w.n_sweeps * Ls[0] ** 3)
    # replicas per size so that all sizes together take ~target_s on `cores` threads
    att_budget = target_s * cores / per_att
    per_size = att_budget / len(Ls)
    tasks = []
    for L in Ls:
        n = max(1, int(per_size / (w.n_sweeps * L ** 3)))
        n = min(n, w.n_rep)
        tasks += [(L, r) for r in range(n)]

    def one(task):
        L, r = task
        oracle.sa_run(L, inst[L][0], w.seed, specs[L].chain, thr_h, n_rep=1, rep0=r)
        return w.n_sweeps * L ** 3

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        attempts = sum(ex.map(one, tasks))
    dt = time.perf_counter() - t0
    counts = {L: sum(1 for t in tasks if t[0] == L) for L in Ls}
    sample = ", ".join(f"L={L}: {counts[L]} replicas" for L in Ls)
    return {"value": attempts / dt, "unit": "spin-flip attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"first instance of each size, {sample}, {w.n_sweeps} sweeps each "
                      f"({attempts:.3g} attempts in {dt:.1f} s)"}


def cpu_baseline_fragment(sg, wl, L=12):
    """The oracle's fragment decimation of L = 12 instances of the measured
    workload (first setting), one instance per host thread."""
    import concurrent.futures as cf

    import oracle
    st = wl.fragment_settings()[0]
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    thr = oracle.thresholds(oracle.schedule(0, st.beta0, st.beta1, st.n_sweeps), sg.SG_K_MAX)
    specs = wl.fragment_instances(L, cores)
    Js = [oracle.make_instance(L, s.cls, s.seed)[0] for s in specs]
    seed = wl.philox_seed("fragment")

    def one(k):
        oracle.frag_decimate(L, Js[k], st.core, st.halo, st.replicas, seed, k, thr, order=st.order)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(cores)))
    dt = time.perf_counter() - t0
    proposals = cores * (L ** 3 // st.core ** 3) * st.replicas * (st.core + 2 * st.halo) ** 3 * st.n_sweeps
    return {"value": cores / dt, "unit": f"instances/s at L={L} ({st.name})", "cores": cores, "kind": "oracle",
            "proposals_per_s": proposals / dt,
            "sample": f"{cores} instances at L={L}, one per thread, {dt:.1f} s"}


def cpu_baseline_tn(sg, wl, L=20, n_sites=960):
    """The oracle's exact fragment marginals (l = 5, beta = 2) for a sample
    of sites of the first L = 20 instance: random sites whose tables fit the
    LDS tier (the oracle's elimination order makes the larger ones take
    minutes each), with the decimated state of the GPU's own run as the
    fixed spins, one site per task on the host threads."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from oracle import tn
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    spec = wl.tn_instances(L, 1)[0]
    J, _, _ = sg.make_instance(L, spec.cls, spec.seed)
    J = np.asarray(J).reshape(6, L ** 3)
    plan = sg.TnPlan(L, 2, 1)
    dec = sg.tn_decimate(plan, torch.from_numpy(J).cuda(), 2.0, want_score=False)[0].cpu().numpy()[0]
    shapes, _, items = plan.program()
    light = [int(site) for site, s in items if shapes[s][0] <= plan.info()["lds_max_bits"]]
    rng = np.random.default_rng(7)
    sites = [int(i) for i in rng.choice(light, n_sites, replace=False)]
    ph = tn.phases(1, L, 2)

    def one(i):
        return tn.site_score(L, J, tn.fixed_before(dec, ph, i), i, 2, 2.0)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, sites))
    dt = time.perf_counter() - t0
    return {"value": n_sites / dt, "unit": f"site marginals/s at L={L}, l=5 (LDS-tier sites)", "cores": cores,
            "kind": "oracle", "sample": f"{n_sites} random LDS-tier sites of one L={L} instance in {dt:.1f} s"}


def cpu_baseline_pticm(sg, wl, steps=5000):
    """The oracle's PT with cluster moves on the measured workload's instance
    and ladder (L = 12, 2 x 4 walkers, beta 0.2 -> 2.0, moves on every slot),
    one run of `steps` steps per host thread."""
    import concurrent.futures as cf

    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    T = 4
    J, _, _ = oracle.make_instance(12, 6, wl.instance_seed("pt", 12))
    beta = oracle.schedule(1, 0.2, 2.0, T)
    thr = oracle.thresholds(beta, sg.SG_K_MAX)
    # exchange tables up to their last nonzero entry
    full = oracle.exchange_thresholds(beta, 4096)
    M = int(max(np.nonzero(row)[0].max() + 1 if row.any() else 1 for row in full))
    thrx = oracle.exchange_thresholds(beta, M)
    seed = wl.philox_seed("pt")

    def one(r):
        oracle.pticm_run(12, J, seed, r, thr, thrx, steps, icm_from=0)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(cores)))
    dt = time.perf_counter() - t0
    att = cores * steps * 2 * T * 12 ** 3
    return {"value": att / dt, "unit": "spin-flip attempts/s (with cluster moves)", "cores": cores,
            "kind": "oracle", "sample": f"{cores} runs x {steps} steps, one per thread, {dt:.1f} s"}


def cpu_baseline_pt(sg, wl, steps=3000):
    """The oracle's PT on the measured workload's instance and ladder (L = 12,
    32 temperatures, beta 0.2 -> 3.0), one run of `steps` steps per host
    thread."""
    import concurrent.futures as cf

    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    w = wl.pt()
    L, T = w.instance.L, w.T
    J, _, _ = oracle.make_instance(L, 6, w.instance.seed)
    beta = oracle.schedule(1, w.beta0, w.beta1, T)
    thr = oracle.thresholds(beta, sg.SG_K_MAX)
    full = oracle.exchange_thresholds(beta, 4096)
    M = int(max(np.nonzero(row)[0].max() + 1 if row.any() else 1 for row in full))
    thrx = oracle.exchange_thresholds(beta, M)

    def one(r):
        oracle.pt_run(L, J, w.seed, r, thr, thrx, steps)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(cores)))
    dt = time.perf_counter() - t0
    att = cores * steps * T * L ** 3
    return {"value": att / dt, "unit": "spin-flip attempts/s", "cores": cores,
            "kind": "oracle", "sample": f"{cores} runs x {steps} steps, one per thread, {dt:.1f} s"}


# ---------------------------------------------------------------------------

def select_shapes(a, sg, Ls, n_sweeps):
    """Launch shapes per lattice size: fixed by --variants, else autotuned on
    the device before the timed region (timed at the workload's sweep count,
    so per-group set-up weighs as it will)."""
    tuning = {}
    if a.variants:
        for item in a.variants.split(","):
            L, v = (int(x) for x in item.split("="))
            if L in Ls:
                sg.select_variant(L, v)
                tuning[L] = {"variant": v, **sg.sa_variants(L)[v], "fixed": True}
    elif not a.no_autotune:
        for L in sorted(Ls):
            res = sg.autotune(L, n_rep=16384 if L <= 16 else 4096, n_sweeps=n_sweeps, repeats=2)
            v = res["selected"]
            tuning[L] = {"variant": v, **sg.sa_variants(L)[v],
                         "candidates_ms": [round(r["ms"], 4) for r in res["results"]]}
            log(f"autotune L={L}: variant {v} {tuning[L]}")
    return tuning


def run_sa_batch(a, sg, wl, torch, stream, steps, warmup, with_cpu):
    """The 48-instance batched workload (L = 8/12/16, 1024 replicas, 256
    sweeps); returns its bench record."""
    tuning = select_shapes(a, sg, {s.L for s in wl.sa_batch().instances}, wl.sa_batch().n_sweeps)
    # direct launches: per-kernel timing events are recorded on each branch
    w, insts, jobs, batch, thr_h, t_host, E_all = build_sa_batch(sg, wl, torch, graph=False)
    egs = torch.tensor([i.E_gs for i in insts], dtype=torch.int64, device="cuda")
    info = batch.info()
    attempts = info["attempts"]
    log(f"sa_batch: {len(insts)} instances, {info['kernels']} kernels, {info['groups']} groups, "
        f"{attempts:.4g} attempts/step; host set-up {t_host:.2f} s")
    eps = {}

    ka = torch.cuda.Event(enable_timing=True)
    kb = torch.cuda.Event(enable_timing=True)

    def step():
        ka.record(stream)
        batch.launch(stream)          # forks onto one stream per L, joins back
        kb.record(stream)
        run_eps(sg, E_all, egs, eps, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kernel_ms = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    launch_ms = []
    for _ in range(steps):
        step()
        # device times of this step's batched launch (span of the three
        # concurrent kernels) and of each kernel on its branch stream
        torch.cuda.synchronize()
        launch_ms.append(ka.elapsed_time(kb))
        for k in batch.kernels():
            kernel_ms.setdefault(k["L"], []).append(k["ms"])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    ms_per_step = dev_ms / steps
    value = attempts / (ms_per_step * 1e-3)

    graph_ms = None
    if not a.no_graph_compare:
        gbatch = sg.Batch(jobs, graph=True)

        def gstep():
            gbatch.launch(stream)
            run_eps(sg, E_all, egs, eps, stream)
        for _ in range(warmup):
            gstep()
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(steps):
            gstep()
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / steps
        gbatch.close()

    # quality (not timed): gap statistics of the last step
    st = eps["st"]
    mean_eps = sg.mean_epsilon(st, egs)
    n_le = st["n_le"].cpu().numpy()
    eps_min = (st["emin"].cpu().numpy().astype(np.int64) - egs.cpu().numpy()) / np.abs(egs.cpu().numpy())
    kern = batch.kernels()
    # the dominant launch: the three concurrent k_sa kernels of the batch
    span_ms = float(np.mean(launch_ms))
    achieved = attempts * OPS_PER_ATTEMPT / (span_ms * 1e-3)
    traffic = measured_traffic("sa_batch")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU32_PEAK / 1e12,
                "unit": "T 32-bit VALU ops/s", "frac": achieved / VALU32_PEAK,
                "traffic": None if traffic is None else traffic["bytes_per_launch"],
                "kernel": "k_sa batched launch (3 concurrent kernels, L=8/12/16)",
                "launch_ms": span_ms, "ops_per_attempt": OPS_PER_ATTEMPT,
                "attempts_per_launch": attempts, "kernel_source_hash": kernel_source_hash()}
    out = {
        "metric": "spin-flip attempts/s (batched SA, 48 instances L=8/12/16 x 1024 replicas x 256 sweeps)",
        "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int8", "data": "synthetic",
        "config": {"workload": "sa_batch: 16 tile-planted T6 instances at each of L=8,12,16, "
                               "1024 replicas, 256 sweeps, beta linear 0.1->3.0",
                   "instances": len(insts), "replicas": w.n_rep, "sweeps": w.n_sweeps,
                   "attempts_per_step": attempts, "launch": "3 kernels (one per L) on parallel streams"},
        "graph_replay": None if graph_ms is None else {"ms_per_step": graph_ms,
                                                       "attempts_per_s": attempts / (graph_ms * 1e-3)},
        "roofline": roofline,
        "kernels": [{"L": k["L"], "ms": float(np.mean(kernel_ms[k["L"]])), "attempts": k["attempts"],
                     "attempts_per_s_while_concurrent": k["attempts"] / (float(np.mean(kernel_ms[k["L"]])) * 1e-3)}
                    for k in kern],
        "eps": {"mean": float(mean_eps.mean()), "min": float(eps_min.min()),
                "frac_le_1pct": float(n_le[:, 0].sum() / (n_le.shape[0] * w.n_rep)),
                "frac_le_3pct": float(n_le[:, 1].sum() / (n_le.shape[0] * w.n_rep))},
        "host_setup_s": t_host, "wall_s": wall, "launch_shapes": tuning,
    }
    if with_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_sa(w, thr_h, a.cpu_seconds)
    batch.close()
    return out


def cpu_baseline_uneven(jobs_spec, host, seed, thr_h, target_s):
    """The oracle, unchanged, on replica 0 of a sample of the uneven batch's
    jobs (every m-th job, m chosen so the sample takes about target_s on the
    host threads), one chain per task."""
    import concurrent.futures as cf

    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    # calibrate on one short chain
    j0 = jobs_spec[0]
    t0 = time.perf_counter()
    oracle.sa_run(j0.inst.L, host[0][0], seed, j0.inst.chain, thr_h[j0.n_sweeps], n_rep=1)
    per_att = (time.perf_counter() - t0) / (j0.n_sweeps * j0.inst.L ** 3)
    mean_att = float(np.mean([j.n_sweeps * j.inst.L ** 3 for j in jobs_spec]))
    n_sample = int(max(16, min(len(jobs_spec), target_s * cores / (per_att * mean_att))))
    stride = max(1, len(jobs_spec) // n_sample)
    idx = list(range(0, len(jobs_spec), stride))

    def one(k):
        j = jobs_spec[k]
        oracle.sa_run(j.inst.L, host[k][0], seed, j.inst.chain, thr_h[j.n_sweeps], n_rep=1)
        return j.n_sweeps * j.inst.L ** 3
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        attempts = sum(ex.map(one, idx))
    dt = time.perf_counter() - t0
    return {"value": attempts / dt, "unit": "spin-flip attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"replica 0 of every {stride}-th job of the uneven batch ({len(idx)} jobs, all six L and "
                      f"four budgets; {attempts:.3g} attempts in {dt:.1f} s)"}


def run_uneven(a, sg, wl, torch, stream):
    """The uneven batch (the largest single-GPU workload): 4096 instances of
    mixed L and sweep budget, one captured hipGraph per step plus the
    per-instance gap statistics."""
    import concurrent.futures as cf
    jobs_spec = wl.uneven()
    seed = wl.uneven_seed()
    n_rep = jobs_spec[0].n_rep
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(16) as ex:
        host = list(ex.map(lambda j: sg.make_instance(j.inst.L, j.inst.cls, j.inst.seed), jobs_spec))
    budgets = sorted({j.n_sweeps for j in jobs_spec})
    thr_h = {S: sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S)) for S in budgets}
    thr = {S: sg.to_device_u32(t) for S, t in thr_h.items()}
    insts = [sg.Instance(j.inst.L, h[0], h[2], j.inst.chain) for j, h in zip(jobs_spec, host)]
    t_host = time.perf_counter() - t0
    Ls = sorted({j.inst.L for j in jobs_spec})
    tuning = select_shapes(a, sg, Ls, 256)
    E_all = torch.empty((len(jobs_spec), n_rep), dtype=torch.int32, device="cuda")
    egs = torch.tensor([i.E_gs for i in insts], dtype=torch.int64, device="cuda")
    jobs = [sg.SAJob(inst, thr[j.n_sweeps], j.n_rep, seed, energy=E_all[k])
            for k, (inst, j) in enumerate(zip(insts, jobs_spec))]
    batch = sg.Batch(jobs, graph=True)
    info = batch.info()
    attempts = info["attempts"]
    log(f"uneven: {len(jobs)} jobs, {info['kernels']} kernels, {info['groups']} groups, {attempts:.4g} "
        f"attempts/step; host set-up {t_host:.2f} s")
    targets = (0.01, 0.03, 0.05)
    res = {}

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]

    def step(i=None):
        if i is not None:
            evs[i][0].record(stream)
        batch.launch(stream)
        if i is not None:
            evs[i][1].record(stream)
        res["st"] = sg.epsilon_stats(E_all, egs, targets=targets, eps_max=0.1, n_bins=100, stream=stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(a.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / a.steps
    span_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    value = attempts / (ms_per_step * 1e-3)

    # quality (not timed): per-instance mean gap from the exact energy sums
    st = res["st"]
    mean_eps = sg.mean_epsilon(st, egs)
    n_le = st["n_le"].cpu().numpy()
    hist = st["hist"].cpu().numpy().astype(np.int64).sum(axis=0)
    Lk = np.array([j.inst.L for j in jobs_spec])
    Sk = np.array([j.n_sweeps for j in jobs_spec])
    quality = {str(L): {str(S): {"mean_eps": float(mean_eps[(Lk == L) & (Sk == S)].mean()),
                                 "frac_le_1pct": float(n_le[(Lk == L) & (Sk == S), 0].sum() /
                                                       (n_rep * np.sum((Lk == L) & (Sk == S))))}
                        for S in budgets} for L in Ls}

    # per-kernel device times: one direct (uncaptured) launch of the same plan
    direct = sg.Batch(jobs, graph=False)
    direct.launch(stream)
    torch.cuda.synchronize()
    direct.launch(stream)
    torch.cuda.synchronize()
    kern = direct.kernels()
    direct.close()

    out_plain = None
    if not a.no_extra:
        # plain per-instance sa_anneal calls on a stratified subset; same
        # counters, so the results must equal the batch's bit for bit (the
        # comparison is at equal eps by construction)
        sub = list(range(0, len(jobs), a.plain_stride))
        outs = {k: (torch.empty_like(jobs[k].spins), torch.empty_like(jobs[k].energy), None) for k in sub}

        def plain_fn():
            for k in sub:
                sg.sa_anneal(insts[k], thr[jobs_spec[k].n_sweeps], n_rep, seed, out=outs[k], stream=stream)
        plain_fn()
        torch.cuda.synchronize()
        p0 = torch.cuda.Event(enable_timing=True)
        p1 = torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        plain_fn()
        p1.record(stream)
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1)
        # the batch's spins of these jobs, recomputed by one more graph launch
        batch.launch(stream)
        torch.cuda.synchronize()
        identical = all(torch.equal(outs[k][0], jobs[k].spins) and torch.equal(outs[k][1], jobs[k].energy)
                        for k in sub)
        sub_att = sum(n_rep * jobs_spec[k].n_sweeps * jobs_spec[k].inst.L ** 3 for k in sub)
        sub_ms_batched = ms_per_step * sub_att / attempts
        out_plain = {"jobs": len(sub), "stride": a.plain_stride, "attempts": sub_att, "ms": pms,
                     "attempts_per_s": sub_att / (pms * 1e-3), "bit_identical_to_batch": bool(identical),
                     "batched_over_plain": value / (sub_att / (pms * 1e-3)),
                     "batched_ms_for_same_jobs": sub_ms_batched}

    achieved = attempts * OPS_PER_ATTEMPT / (span_ms * 1e-3)
    traffic = measured_traffic("uneven")
    counted = measured_valu("uneven")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU32_PEAK / 1e12,
                "unit": "T 32-bit VALU ops/s", "frac": achieved / VALU32_PEAK,
                "traffic": None if traffic is None else traffic["bytes_per_launch"],
                "kernel": f"k_sa batched launch ({info['kernels']} concurrent kernels, one per L, hipGraph)",
                "launch_ms": span_ms, "ops_per_attempt": OPS_PER_ATTEMPT, "attempts_per_launch": attempts,
                "kernel_source_hash": kernel_source_hash()}
    if counted is not None:
        roofline["counted_valu_slots_per_attempt"] = counted["valu_slots_per_attempt"]
        roofline["counted_frac"] = attempts * counted["valu_slots_per_attempt"] / (span_ms * 1e-3) / VALU32_PEAK
    out = {
        "metric": "spin-flip attempts/s (uneven batch: 4096 instances, L in {6,8,10,12,16,20}, 64 replicas, "
                  "128..1024 sweeps; batched vs plain at equal eps)",
        "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": "uneven: 4096 tile-planted T6 instances, L uniform in {6,8,10,12,16,20}, 64 "
                               "replicas each, sweeps uniform in {128,256,512,1024}, beta linear 0.1->3.0, "
                               "autotuned launch shapes, hipGraph-captured",
                   "instances": len(jobs), "replicas": n_rep, "attempts_per_step": attempts,
                   "launch": f"{info['kernels']} kernels (one per L) on parallel branches of one hipGraph, "
                             "then epsilon_stats"},
        "plain": out_plain,
        "roofline": roofline,
        "kernels": [{"L": k["L"], "ms": k["ms"], "attempts": k["attempts"],
                     "attempts_per_s_while_concurrent": k["attempts"] / (k["ms"] * 1e-3) if k["ms"] > 0 else None}
                    for k in kern],
        "eps": {"mean": float(mean_eps.mean()), "frac_le_1pct": float(n_le[:, 0].sum() / n_le.shape[0] / n_rep),
                "frac_le_3pct": float(n_le[:, 1].sum() / n_le.shape[0] / n_rep),
                "hist_0_to_10pct_by_0p1pct": hist.tolist(), "by_L_and_sweeps": quality},
        "host_setup_s": t_host, "wall_s": wall, "launch_shapes": tuning,
    }
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_uneven(jobs_spec, host, seed, thr_h, a.cpu_seconds)
    batch.close()
    return out


def main():
    a = parse()
    if a.hw_queues is None and a.workload in ("serve", "uneven"):
        # one stream per lattice size: enough hardware queues let their
        # kernels run side by side (the uneven batch has six sizes)
        a.hw_queues = 16 if a.workload == "serve" else 8
    if a.hw_queues:
        # must be set before HIP starts
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, a.hw_queues))
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import paper_2501_17267_amd as sg
    from paper_2501_17267_amd import workloads as wl
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if a.workload == "uneven":
        out = run_uneven(a, sg, wl, torch, stream)
        if not a.no_extra:
            log("sa_batch leg ...")
            out["sa_batch"] = run_sa_batch(a, sg, wl, torch, stream, steps=max(3, a.steps // 2),
                                           warmup=1, with_cpu=False)
        print(json.dumps(out))
        return
    if a.workload == "sa_batch":
        print(json.dumps(run_sa_batch(a, sg, wl, torch, stream, a.steps, a.warmup, not a.no_cpu_baseline)))
        return

    from paper_2501_17267_amd import benchmarks
    out = benchmarks.run(a.workload, a, sg, wl, torch)
    if a.workload == "fragment" and not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_fragment(sg, wl)
    if a.workload == "pt" and not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_pt(sg, wl)
    if a.workload == "pticm" and not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_pticm(sg, wl)
    if a.workload == "tn" and not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_tn(sg, wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
