"""Optimality gap and time of the linear-time meta-heuristic (Sec. I) versus
system size: eps_lin(L) with the fit a/L + b of Sec. II, and the time per
instance with a fit T = a N^alpha (linear time means alpha -> 1 once the
device is full).

For every L: 20 tile-planted stand-in instances, one decimation each per
setting (workloads.fragment_settings), timed from launch to completion with
the instance already on the device.
"""
from __future__ import annotations

import time

import numpy as np

from . import Instance, epsilon, fragment_decimate, make_schedule, make_thresholds, to_device_u32
from . import workloads as wl


def run(torch, sizes=(8, 12, 16, 20, 24, 32, 48, 64), n_inst=20, log=print):
    seed = wl.philox_seed("fragment")
    out = {"settings": {}, "sizes": list(sizes), "n_inst": n_inst}
    for st in wl.fragment_settings():
        thr = to_device_u32(make_thresholds(make_schedule(0, st.beta0, st.beta1, st.n_sweeps)))
        per_L = {}
        for L in sizes:
            if L % st.core or st.core + 2 * st.halo >= L:
                continue
            specs = wl.fragment_instances(L, n_inst)
            insts = [Instance.generate(s.L, s.seed, s.chain) for s in specs]
            # warm-up (first launch of the kernel at this shape)
            fragment_decimate(insts[0], thr, st.core, st.halo, st.replicas, st.order, 1, seed)
            torch.cuda.synchronize()
            ms, eps = [], []
            for k, inst in enumerate(insts):
                t0 = time.perf_counter()
                _, en = fragment_decimate(inst, thr, st.core, st.halo, st.replicas, st.order, 1, seed, run0=k)
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1e3)
                eps.append(float(epsilon(en, inst.E_gs).cpu().numpy()[0]))
            # all instances at once on one stream each after the other is the
            # plain form; the throughput form puts 20 runs of one instance in
            # one call
            t0 = time.perf_counter()
            fragment_decimate(insts[0], thr, st.core, st.halo, st.replicas, st.order, n_inst, seed)
            torch.cuda.synchronize()
            batch_ms = (time.perf_counter() - t0) * 1e3
            proposals = (L ** 3 // st.core ** 3) * st.replicas * (st.core + 2 * st.halo) ** 3 * st.n_sweeps
            e = np.array(eps)
            per_L[L] = {"N": L ** 3, "ms_mean": float(np.mean(ms)), "ms_max": float(np.max(ms)),
                        "eps_mean": float(e.mean()), "eps_max": float(e.max()),
                        "frac_exact": float(np.mean(e == 0.0)),
                        "runs_per_call_ms": batch_ms / n_inst,
                        "proposals_per_s_single": proposals / (np.mean(ms) * 1e-3),
                        "proposals_per_s_20_runs": n_inst * proposals / (batch_ms * 1e-3)}
            log(f"fragment {st.name} L={L}: {per_L[L]}")
        Ls = np.array(sorted(per_L), np.float64)
        fit = {}
        if len(Ls) >= 3:
            em = np.array([per_L[int(L)]["eps_mean"] for L in Ls])
            A = np.stack([1.0 / Ls, np.ones_like(Ls)], axis=1)
            (a, b), *_ = np.linalg.lstsq(A, em, rcond=None)
            fit["eps_a_over_L_plus_b"] = {"a": float(a), "b": float(b)}
            for lo, key in ((0, "time_alpha_all"), (24, "time_alpha_L_ge_24")):
                sel = Ls >= lo
                if sel.sum() >= 2:
                    N = Ls[sel] ** 3
                    T = np.array([per_L[int(L)]["ms_mean"] for L in Ls[sel]])
                    fit[key] = float(np.polyfit(np.log(N), np.log(T), 1)[0])
        out["settings"][st.name] = {"core": st.core, "halo": st.halo, "replicas": st.replicas,
                                    "n_sweeps": st.n_sweeps, "order": st.order,
                                    "beta": [st.beta0, st.beta1],
                                    "per_L": {str(L): v for L, v in per_L.items()}, "fits": fit}
    return out
