"""Secondary benchmark modes of bench.py (one JSON object each).

  microbench  VALU instruction throughput probes (the ALU ceiling's inputs)
  sa_small    one L=4 instance, 64 restarts x 1000 sweeps
  plain       the batched-SA workload issued as 48 separate sa_anneal calls
  pt          parallel tempering: L=12, 32 temperatures, 128 runs x 2000 steps
  uneven      4096 instances of mixed L and sweep budget: batch vs plain calls
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

N_CU = 256
CLOCK_HZ = 2.4e9
VALU32_PEAK = N_CU * 64 * CLOCK_HZ


def _time(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def microbench(a, sg, wl, torch):
    lib = sg.lib()
    lib.sg_microbench_valu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]
    lib.sg_microbench_valu.restype = ctypes.c_int
    stream = torch.cuda.current_stream()
    blocks, iters = 256 * 16, 4096
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    names = ["v_mad_u64_u32", "xor3", "add3", "bitfield select"]
    res = {}
    for op in range(4):
        def fn():
            rc = lib.sg_microbench_valu(op, blocks, iters, out.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
            assert rc == 0
        ms = _time(torch, fn, 5, 2, stream)
        instr = blocks * 256 * iters * 8.0
        rate = instr / (ms * 1e-3)
        res[names[op]] = {"lane_ops_per_s": rate, "frac_of_full_rate": rate / VALU32_PEAK,
                          "ms": ms}
    return {"metric": "VALU instruction throughput", "unit": "lane-ops/s",
            "peak_full_rate": VALU32_PEAK, "probes": res}


def copy(a, sg, wl, torch):
    """A 256 MiB device-to-device copy with the library's plain copy kernel."""
    lib = sg.lib()
    lib.sg_microbench_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.sg_microbench_copy.restype = ctypes.c_int
    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()

    def fn():
        rc = lib.sg_microbench_copy(src.data_ptr(), dst.data_ptr(), nbytes, ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    assert bool((dst == 1).all())
    return {"metric": "device copy bandwidth", "bytes_read": nbytes, "bytes_written": nbytes,
            "ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}


def sa_small(a, sg, wl, torch):
    w = wl.sa_small()
    spec = w.instances[0]
    inst = sg.Instance.generate(spec.L, spec.seed, spec.chain)
    thr = sg.to_device_u32(sg.make_thresholds(sg.make_schedule(w.kind, w.beta0, w.beta1, w.n_sweeps)))
    stream = torch.cuda.current_stream()
    res = {}

    def fn():
        res["out"] = sg.sa_anneal(inst, thr, w.n_rep, w.seed)
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    att = w.n_rep * w.n_sweeps * spec.L ** 3
    eps = sg.epsilon(res["out"][1], inst.E_gs).cpu().numpy()
    return {"metric": "spin-flip attempts/s (L=4, 64 restarts x 1000 sweeps)", "value": att / (ms * 1e-3),
            "unit": "spin-flip attempts/s", "ms_per_step": ms, "eps_mean": float(eps.mean()),
            "eps_min": float(eps.min()), "frac_at_gs": float(np.mean(eps == 0.0))}


def plain(a, sg, wl, torch):
    """The batched workload as 48 plain per-instance calls on one stream."""
    w = wl.sa_batch()
    beta = sg.make_schedule(w.kind, w.beta0, w.beta1, w.n_sweeps)
    thr = sg.to_device_u32(sg.make_thresholds(beta))
    insts = [sg.Instance.generate(s.L, s.seed, s.chain) for s in w.instances]
    outs = [(torch.empty((w.n_rep, i.L ** 3), dtype=torch.int8, device="cuda"),
             torch.empty(w.n_rep, dtype=torch.int32, device="cuda"), None) for i in insts]
    stream = torch.cuda.current_stream()

    def fn():
        for inst, o in zip(insts, outs):
            sg.sa_anneal(inst, thr, w.n_rep, w.seed, out=o)
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    att = sum(w.n_rep * w.n_sweeps * i.L ** 3 for i in insts)
    return {"metric": "spin-flip attempts/s (48 plain sa_anneal calls)", "value": att / (ms * 1e-3),
            "unit": "spin-flip attempts/s", "ms_per_step": ms}


def pt(a, sg, wl, torch):
    w = wl.pt()
    inst = sg.Instance.generate(w.instance.L, w.instance.seed, 0)
    beta = sg.make_schedule(1, w.beta0, w.beta1, w.T)
    thr = sg.to_device_u32(sg.make_thresholds(beta))
    M = sg.exchange_table_width(beta)
    thrx = sg.to_device_u32(sg.make_exchange_thresholds(beta, M))
    stream = torch.cuda.current_stream()
    res = {}

    groups = getattr(a, "pt_groups", 0)
    ws = None
    if groups != 1:
        ws = torch.empty((sg.pt_split_workspace_bytes(w.n_runs, w.T) + 7) // 8, dtype=torch.int64, device="cuda")

    def fn():
        res["out"] = sg.pt_run(inst, thr, thrx, w.n_runs, w.n_steps, w.seed, want_trace=True, groups=groups,
                               workspace=ws, check=False)
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    if ws is not None and int(ws.view(torch.int32)[0].item()) != 0:
        raise RuntimeError("pt: a work group gave up waiting on another (status word set)")
    att = w.n_runs * w.n_steps * w.T * w.instance.L ** 3
    final_min = res["out"]["emin_trace"][:, -1].cpu().numpy().astype(np.int64)
    eps = (final_min - inst.E_gs) / abs(inst.E_gs)
    rate = att / (ms * 1e-3)
    ops = 20   # VALU lane-slots per attempt in the model of the SA bench line
    peak = 256 * 4 * 16 * 2.4e9 / 1e12
    return {"metric": "spin-flip attempts/s (PT L=12, T=32, 128 runs x 2000 steps)",
            "value": rate, "unit": "spin-flip attempts/s", "ms_per_step": ms,
            "roofline": {"bound": "alu", "achieved": ops * rate / 1e12, "peak": peak,
                         "unit": "T 32-bit VALU ops/s", "frac": ops * rate / 1e12 / peak,
                         "note": ("one work group per run: 128 runs occupy 128 of the 256 CUs" if groups == 1 else
                                  "each run spread over work groups (sg_pt_run_split) so that the launch "
                                  "fills the 256 CUs")},
            "pt_groups": "auto" if groups == 0 else groups,
            "exchange_attempts_per_step": w.n_runs * w.n_steps * (w.T - 1) / 2,
            "eps_best_mean": float(eps.mean()), "eps_best_min": float(eps.min())}


def _make_instances(sg, specs, threads=16):
    """Host-generate instances in parallel (the generator releases the GIL)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda s: sg.make_instance(s.L, s.cls, s.seed), specs))


def uneven(a, sg, wl, torch):
    """4096 instances of mixed L and sweep budget: one graph-replayed batch
    against per-instance sa_anneal calls (timed on a stratified subset)."""
    jobs_spec = wl.uneven()
    seed = wl.uneven_seed()
    t0 = time.perf_counter()
    host = _make_instances(sg, [j.inst for j in jobs_spec])
    budgets = sorted({j.n_sweeps for j in jobs_spec})
    thr = {S: sg.to_device_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S))) for S in budgets}
    insts = [sg.Instance(j.inst.L, h[0], h[2], j.inst.chain) for j, h in zip(jobs_spec, host)]
    t_host = time.perf_counter() - t0
    tuning = {}
    if not getattr(a, "no_autotune", False):
        for L in sorted({j.inst.L for j in jobs_spec}):
            res = sg.autotune(L, n_rep=8192, n_sweeps=256, repeats=2)
            tuning[L] = res["selected"]
    jobs = [sg.SAJob(inst, thr[j.n_sweeps], j.n_rep, seed) for inst, j in zip(insts, jobs_spec)]
    batch = sg.Batch(jobs, graph=True)
    info = batch.info()
    stream = torch.cuda.current_stream()
    ms = _time(torch, lambda: batch.launch(stream), a.steps, a.warmup, stream)
    attempts = info["attempts"]
    # plain per-instance launches on a stratified subset (every 32nd job)
    sub = list(range(0, len(jobs_spec), 32))
    outs = {k: (torch.empty_like(jobs[k].spins), torch.empty_like(jobs[k].energy), None) for k in sub}

    def plain_fn():
        for k in sub:
            sg.sa_anneal(insts[k], thr[jobs_spec[k].n_sweeps], jobs_spec[k].n_rep, seed, out=outs[k])
    pms = _time(torch, plain_fn, 1, 1, stream)
    sub_att = sum(jobs_spec[k].n_rep * jobs_spec[k].n_sweeps * jobs_spec[k].inst.L ** 3 for k in sub)
    identical = all(torch.equal(outs[k][0], jobs[k].spins) and torch.equal(outs[k][1], jobs[k].energy)
                    for k in sub)
    eps_by_L = {}
    for inst, job in zip(insts, jobs):
        e = sg.epsilon(job.energy, inst.E_gs)
        eps_by_L.setdefault(inst.L, []).append(e)
    eps_stats = {L: {"mean": float(torch.cat(v).mean()), "frac_le_1pct": float((torch.cat(v) <= 0.01).double().mean())}
                 for L, v in sorted(eps_by_L.items())}
    batch.close()
    return {"metric": "spin-flip attempts/s (uneven batch: 4096 instances, L in {6..20}, 64 replicas, "
                      "128..1024 sweeps)",
            "value": attempts / (ms * 1e-3), "unit": "spin-flip attempts/s", "ms_per_step": ms,
            "attempts_per_step": attempts, "kernels": info["kernels"], "groups": info["groups"],
            "plain_subset": {"instances": len(sub), "attempts": sub_att, "ms": pms,
                             "attempts_per_s": sub_att / (pms * 1e-3)},
            "batched_over_plain": (attempts / (ms * 1e-3)) / (sub_att / (pms * 1e-3)),
            "bit_identical_batch_vs_plain": identical, "eps_by_L": eps_stats,
            "launch_shapes": tuning, "host_setup_s": t_host}


def serve(a, sg, wl, torch):
    """Poisson stream of anneal requests through the continuous-batching server."""
    from . import serving
    import sys
    dur = float(getattr(a, "duration", 60.0))
    res = serving.run_poisson(torch, rate=float(getattr(a, "rate", 2000.0)), duration=dur,
                              warmup=min(10.0, dur / 6), seed=wl.philox_seed("serve") & 0xFFFF,
                              pool=4, chunk=int(getattr(a, "chunk", 512)),
                              chunk_attempts=int(getattr(a, "chunk_attempts", 1 << 24)),
                              log=lambda *m: print("[serve]", *m, file=sys.stderr, flush=True))
    res["metric"] = ("served spin-flip attempts/s and latency (Poisson 2000 req/s, L even 8..32 "
                     "+ 5% L=64, sweeps log-uniform 64..4096, one replica per request)")
    res["value"] = res["attempts_per_s"]
    import os
    res["hw_queues"] = os.environ.get("GPU_MAX_HW_QUEUES", "default")
    res["unit"] = "spin-flip attempts/s"
    return res


def tteps(a, sg, wl, torch):
    """Time-to-eps at eps = 1% (and 3%, 5%) versus N, plain / batched / served."""
    from . import tteps as tt
    import sys
    res = tt.run(torch, log=lambda *m: print("[tteps]", *m, file=sys.stderr, flush=True))
    res["metric"] = "TT-eps at eps = 1% (3%, 5%) vs N; plain, batched and served forms"
    return res


def fragment(a, sg, wl, torch):
    """eps_lin and time per instance of the linear-time meta-heuristic vs L."""
    from . import fragment as fr
    import sys
    res = fr.run(torch, log=lambda *m: print("[fragment]", *m, file=sys.stderr, flush=True))
    res["metric"] = "eps_lin and time per instance of the fragment meta-heuristic vs L"
    return res


def fragment_call(a, sg, wl, torch):
    """One 20-run decimation call of the measured fragment setting at L = 32
    (after one warm-up call): the unit the fragment kernel's counters are
    taken on."""
    st = wl.fragment_settings()[0]
    L, n_runs = 32, 20
    thr = sg.to_device_u32(sg.make_thresholds(sg.make_schedule(0, st.beta0, st.beta1, st.n_sweeps)))
    spec = wl.fragment_instances(L, 1)[0]
    inst = sg.Instance.generate(L, spec.seed, spec.chain)
    seed = wl.philox_seed("fragment")
    sg.fragment_decimate(inst, thr, st.core, st.halo, st.replicas, st.order, n_runs, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, en = sg.fragment_decimate(inst, thr, st.core, st.halo, st.replicas, st.order, n_runs, seed)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    nominal = n_runs * (L ** 3 // st.core ** 3) * st.replicas * (st.core + 2 * st.halo) ** 3 * st.n_sweeps
    return {"metric": "ms of one 20-run fragment decimation call (L = 32, l = 5, 8 anneals x 100 sweeps)",
            "ms": ms, "nominal_proposals_per_s": nominal / (ms * 1e-3),
            "eps_mean": float(((en.cpu().numpy().astype(np.int64) - inst.E_gs) / abs(inst.E_gs)).mean())}


def tn(a, sg, wl, torch):
    """The tensor-network subsystem optimiser (exact l = 5 fragment
    marginals at beta = 2): eps_lin and time vs L, beta and l studies."""
    from . import tn_study
    import sys
    res = tn_study.run(torch, log=lambda *m: print("[tn]", *m, file=sys.stderr, flush=True))
    res["metric"] = "eps_lin and time per instance of the tensor-network meta-heuristic vs L"
    return res


def wide(a, sg, wl, torch):
    """One anneal of few replicas of L = 32 and 64 (256 sweeps): the
    multi-work-group path that sa_anneal picks by itself, against the
    single-work-group kernel of the same size; results are identical."""
    out = {"metric": "ms per anneal of few replicas, wide path vs one work group per replica group", "rows": []}
    thr = sg.to_device_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 256)))
    for L in (32, 64):
        inst = sg.Instance.generate(L, wl.instance_seed("sa_batch", 64000 + L), chain=1)
        for n in (1, 16):
            res = {}
            for name in ("wide", "group"):
                def fn():
                    if name == "wide":
                        return sg.sa_anneal(inst, thr, n, 5)
                    return sg.sa_anneal_variant(inst, thr, n, 5, sg.selected_variant(L))
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(a.steps):
                    r = fn()
                torch.cuda.synchronize()
                res[name] = ((time.perf_counter() - t0) * 1e3 / a.steps, r[1])
            out["rows"].append({"L": L, "replicas": n, "wide_ms": res["wide"][0], "group_ms": res["group"][0],
                                "identical": bool(torch.equal(res["wide"][1], res["group"][1]))})
    return out


def large(a, sg, wl, torch):
    """The large-lattice path at a replica count that fills the device: 256
    replicas of one instance at L = 32 (spins in LDS, couplings streamed from
    the encoded image) and at L = 64 (spins in the workspace too), 256 sweeps,
    one work group per replica group, the launch shape autotuned at that
    replica count; and one replica of each on the wide path (one launch per
    colour phase).  Rooflines: the 20-slot VALU model against 39.3 T
    lane-ops/s, and, where the spins live in the workspace, HBM against
    8 TB/s at 5 B per attempt (couplings read once per bond, a spin read and
    written once per sweep); `frac` is taken against the lower of the ones
    that apply, the binding one."""
    out = {"metric": "spin-flip attempts/s of the large-lattice kernels (256 replicas x 256 sweeps)", "rows": []}
    S, R = 256, 256
    thr = sg.to_device_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S)))
    stream = torch.cuda.current_stream()
    valu_roof = VALU32_PEAK / 20
    hbm_roof = 8e12 / 5
    for L in (32, 64):
        inst = sg.Instance.generate(L, wl.instance_seed("sa_batch", 64000 + L), chain=1)
        fixed = dict(tuple(int(x) for x in item.split("=")) for item in (getattr(a, "variants", None) or "").split(",") if item)
        if L in fixed:
            v, cand = fixed[L], None
        else:
            tuned = sg.autotune(L, n_rep=R, n_sweeps=16, repeats=3)
            v, cand = tuned["selected"], [round(r["ms"], 4) for r in tuned["results"]]
        res = {}

        def fn():
            res["out"] = sg.sa_anneal_variant(inst, thr, R, 5, v)
        ms = _time(torch, fn, a.steps, a.warmup, stream)
        att = R * S * L ** 3
        rate = att / (ms * 1e-3)
        one = {}

        def fn1():
            one["out"] = sg.sa_anneal(inst, thr, 1, 5)
        ms1 = _time(torch, fn1, max(2, a.steps // 2), 1, stream)
        # the HBM roof binds only where the spins stream from the workspace
        spins_hbm = bool(sg.sa_variants(L)[v]["spins_in_hbm"])
        roof = min(valu_roof, hbm_roof) if spins_hbm else valu_roof
        out["rows"].append({"L": L, "replicas": R, "sweeps": S, "variant": v, "candidates_ms_16_sweeps": cand,
                            "ms": ms, "attempts_per_s": rate,
                            "valu_frac_20_slot": rate / valu_roof, "hbm_frac_5B": rate / hbm_roof,
                            "binding_roof": "hbm_5B" if roof == hbm_roof else "valu_20_slot",
                            "frac": rate / roof,
                            "one_replica_wide_ms": ms1, "one_replica_us_per_sweep": ms1 * 1e3 / S})
    return out


def tn_call(a, sg, wl, torch):
    """One 20-instance decimation of the tensor-network optimiser's measured
    setting (L = 20, l = 5, beta = 2, wavefront order): ms per call and the
    workspace-tier step's algorithmic bytes per call (8 B per canonical read
    and per written entry), the unit its roofline is taken on."""
    from . import tn_study
    L, n = 20, 20
    plan = sg.TnPlan(L, 2, 1)
    J, egs = tn_study._batch(torch, L, n)
    ws = torch.empty((plan.workspace_bytes(n, True) + 7) // 8, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}

    def fn():
        res["out"] = sg.tn_decimate(plan, J, 2.0, workspace=ws, want_score=False)
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    eps = tn_study._eps(res["out"][1], egs)
    plan.close()
    step_bytes = tn_study.workspace_step_bytes(L, 2, n, 8)
    return {"metric": "ms per 20-instance tensor-network decimation (L = 20, l = 5, beta = 2)", "ms_per_call": ms,
            "ms_per_instance": ms / n, "workspace_step_bytes_per_call": step_bytes,
            "step_bytes_per_s_over_whole_call": step_bytes / (ms * 1e-3), "eps_mean": float(eps.mean())}


def pticm(a, sg, wl, torch):
    """PT with isoenergetic cluster moves at the tuned ladder (L = 12, T = 4
    slots x 2 copies, beta 0.2 -> 2.0, moves on every slot), 128 runs x 200
    steps: spin-flip attempts/s and time per step."""
    inst = sg.Instance.generate(12, wl.instance_seed("pt", 12), chain=0)
    T, runs, steps = 4, 128, 200
    beta = sg.make_schedule(1, 0.2, 2.0, T)
    thr = sg.to_device_u32(sg.make_thresholds(beta))
    M = sg.exchange_table_width(beta)
    thrx = sg.to_device_u32(sg.make_exchange_thresholds(beta, M))
    stream = torch.cuda.current_stream()
    res = {}

    def fn():
        res["out"] = sg.pticm_run(inst, thr, thrx, runs, steps, wl.philox_seed("pt"), icm_from=0, want_icm=True)
    ms = _time(torch, fn, a.steps, a.warmup, stream)
    att = runs * steps * 2 * T * 12 ** 3
    fl = res["out"]["icm_flipped"].float().mean().item()
    rate = att / (ms * 1e-3)
    peak = 256 * 4 * 16 * 2.4e9 / 1e12
    return {"metric": "spin-flip attempts/s (PT+ICM L=12, 2 x 4 walkers, 128 runs x 200 steps)",
            "value": rate, "unit": "spin-flip attempts/s", "ms_per_call": ms,
            "us_per_step": ms * 1e3 / steps, "sites_flipped_per_step_mean": fl,
            "roofline": {"bound": "alu", "achieved": 20 * rate / 1e12, "peak": peak, "unit": "T 32-bit VALU ops/s",
                         "frac": 20 * rate / 1e12 / peak,
                         "note": "Metropolis work only (20 VALU slots per attempt); the cluster moves (one wave "
                                 "per slot, breadth-first rounds on bit-packed double columns) take the rest of a step"}}


def tuning(a, sg, wl, torch):
    """App. D form: SA beta-range grid at L = 10 and PT ladder grid at L = 4
    as the paper prints them, then TT-eps and alpha(eps) at eps = 3, 4, 5 %
    for SA (L = 20..56) and PT with cluster moves (L = 6..12)."""
    from . import tuning as tu
    import sys
    res = tu.run(torch, log=lambda *m: print("[tuning]", *m, file=sys.stderr, flush=True))
    # the table first: alpha(eps) of SA (L = 20..56) and of PT with cluster
    # moves (L = 6..12), plain and batched forms
    return {"metric": "alpha(eps) at eps = 3, 4, 5% after App. D tuning (SA at L = 10, PT at L = 4)",
            "alpha_table": res.pop("alpha_table"), **res}


def pt_tteps(a, sg, wl, torch):
    """PT TT-eps versus N (L = 6..12) at eps = 3, 4, 5 % with the tuned ladder
    (T = 8, beta 0.2 -> 2.0): one run alone (pt_run), one run alone spread
    over work groups (sg_pt_run_split) and 20 runs per launch."""
    from . import tuning as tu
    import sys
    res = tu.pt_tteps(torch, T=8, beta_max=2.0, log=lambda *m: print("[pt_tteps]", *m, file=sys.stderr, flush=True))
    res["metric"] = "PT TT-eps vs N at eps = 3, 4, 5% (plain, split, batched)"
    return res


def run(name, a, sg, wl, torch):
    fn = {"microbench": microbench, "copy": copy, "sa_small": sa_small, "plain": plain, "pt": pt,
          "uneven": uneven, "serve": serve, "tteps": tteps, "fragment": fragment, "fragment_call": fragment_call, "tn": tn, "tuning": tuning, "pt_tteps": pt_tteps,
          "wide": wide, "pticm": pticm, "large": large, "tn_call": tn_call}[name]
    return fn(a, sg, wl, torch)
