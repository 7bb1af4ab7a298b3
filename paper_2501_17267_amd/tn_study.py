"""The paper's own form of the meta-heuristic (Sec. II, App. B, C): the
tensor-network subsystem optimiser (exact l^3 fragment marginals, beta = 2)
on tile-planted stand-in instances.

eps_lin(L)  20 instances per L, l = 5, beta = 2, wavefront order: mean and
            largest eps, the fit a/L + b (Sec. II), the time per instance
            alone and in a 20-instance call, and the table pair updates per
            second; the tropical (zero-temperature) form beside it.
beta study  App. C: mean eps versus beta at one size.
l study     App. B: mean eps versus the fragment edge at L = 20 (l = 3, 5;
            single-spin fragments are centred, so l is odd here).
classes     mean eps of both forms at L = 12, l = 3 and 5, on every stand-in
            tile class (0, 2, 4 or 6 frustrated faces, and mixed tiles).
"""
from __future__ import annotations

import time

import numpy as np

from . import TnPlan, make_instance, tn_decimate
from . import workloads as wl


def workspace_step_bytes(L, h, n_inst, elem, order=1, fused=True):
    """Algorithmic bytes the workspace tier's step kernel moves in one
    decimation of n_inst instances: for every workspace-tier table (both
    centre values) and every round, elem bytes per canonical read (none at
    the first step; two where the eliminated slot is active, twice that
    again where a fused round's second slot is canonical) and per entry the
    round writes (a fused round writes only its second step's entries).
    fused=False counts every step as its own round (beta above
    SG_TN_FUSE_BETA_MAX).  Host only: from the plan's exported programs."""
    plan = TnPlan(L, h, order)
    shapes, steps, items = plan.program()
    shape_rounds, rounds = plan.rounds()
    lds_bits = plan.info()["lds_max_bits"]
    plan.close()
    per_shape = {}
    total = 0
    for _, s in items:
        if int(shapes[s][0]) <= lds_bits:
            continue
        if s not in per_shape:
            per_shape[s] = shape_step_entries(shapes, steps, shape_rounds, rounds, s, fused) * elem
        total += 2 * per_shape[s]
    return total * n_inst


def shape_step_entries(shapes, steps, shape_rounds, rounds, s, fused=True):
    """Entries one table of shape s moves through the workspace tier's
    rounds: canonical reads plus written entries (see workspace_step_bytes)."""
    pc = lambda v: bin(v).count("1")
    ns, s0 = int(shapes[s][1]), int(shapes[s][2])
    rows = ([(t, 0, 0, 0) for t in range(ns)] if not fused else
            [tuple(int(v) for v in rounds[r]) for r in range(shape_rounds[s][0], sum(shape_rounds[s]))])
    n = 0
    for t, fz, read_bits, bcode in rows:
        row = steps[s0 + t]
        a_act, n_base, nm = int(row[8]), int(row[10]), int(row[11]) & 0xFFFFFFFF
        reads = 0 if t == 0 else (2 if a_act else 1)
        if not fz:
            n += (1 << n_base) * (reads + (1 << pc(nm)))
        else:
            nxt = steps[s0 + t + 1]
            bbit, nm1 = 1 << int(nxt[1]), int(nxt[11]) & 0xFFFFFFFF
            reads *= 2 if (bcode & 0xFF) == 1 else 1
            n += (1 << read_bits) * (reads + (1 << (pc(nm & ~bbit) + pc(nm1))))
    return n


def study_step_bytes(sizes=(8, 12, 16, 20, 24, 32), n_inst=20, beta_L=12, n_betas=6, n_classes=5):
    """Algorithmic workspace-step bytes of one run(): (sum-product, tropical).
    Per size: a one-instance warm-up, the timed one-instance and n_inst-instance
    calls (sum-product) and one n_inst call (tropical); the beta study at
    beta_L; the l study at L = 20 (l = 5 is the workspace tier's share); the
    class study at L = 12 with both forms."""
    fp = tr = 0
    for L in sizes:
        fp += workspace_step_bytes(L, 2, 1 + 1 + n_inst, 8)
        tr += workspace_step_bytes(L, 2, n_inst, 4)
    fp += workspace_step_bytes(beta_L, 2, n_betas * n_inst, 8) + workspace_step_bytes(20, 2, n_inst, 8)
    fp += n_classes * workspace_step_bytes(12, 2, n_inst, 8)
    tr += n_classes * workspace_step_bytes(12, 2, n_inst, 4)
    return fp, tr


def _batch(torch, L, n):
    specs = wl.tn_instances(L, n)
    Js, egs = [], []
    for s in specs:
        J, _, e = make_instance(L, s.cls, s.seed)
        Js.append(np.asarray(J).reshape(6, L ** 3))
        egs.append(e)
    return torch.from_numpy(np.stack(Js)).cuda(), np.array(egs, np.int64)


def _eps(en, egs):
    e = en.cpu().numpy().astype(np.int64)
    return (e - egs) / np.abs(egs)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def run(torch, sizes=(8, 12, 16, 20, 24, 32), n_inst=20, beta=2.0, beta_L=12,
        betas=(0.5, 1.0, 2.0, 3.0, 5.0, 8.0), log=print):
    out = {"sizes": list(sizes), "n_inst": n_inst, "beta": beta, "halo": 2, "order": 1, "per_L": {}}
    for L in sizes:
        plan = TnPlan(L, 2, 1)
        info = plan.info()
        J, egs = _batch(torch, L, n_inst)
        ws = torch.empty((plan.workspace_bytes(n_inst, True) + 7) // 8, dtype=torch.float64, device="cuda")
        tn_decimate(plan, J[:1], beta, workspace=ws, want_score=False)          # warm-up
        (sp, en, _), ms1 = _timed(torch, lambda: tn_decimate(plan, J[:1], beta, workspace=ws, want_score=False))
        (sp, en, _), msb = _timed(torch, lambda: tn_decimate(plan, J, beta, workspace=ws, want_score=False))
        eps = _eps(en, egs)
        (_, ent, _), mst = _timed(torch, lambda: tn_decimate(plan, J, 0.0, True, workspace=ws, want_score=False))
        epst = _eps(ent, egs)
        row = {"N": L ** 3, "eps_mean": float(eps.mean()), "eps_max": float(eps.max()),
               "frac_exact": float(np.mean(eps == 0.0)),
               "ms_single": ms1, "ms_per_instance_batched": msb / n_inst,
               "pair_updates_per_instance": info["pair_updates"],
               "pair_updates_per_s_batched": info["pair_updates"] * n_inst / (msb * 1e-3),
               "lds_sites": info["n_lds_sites"], "hbm_sites": info["n_hbm_sites"], "max_bits": info["max_bits"],
               "tropical_eps_mean": float(epst.mean()), "tropical_ms_per_instance_batched": mst / n_inst}
        log(f"tn L={L}: {row}")
        out["per_L"][str(L)] = row
        del ws
        plan.close()
    Ls = np.array(sorted(int(L) for L in out["per_L"]), np.float64)
    if len(Ls) >= 3:
        em = np.array([out["per_L"][str(int(L))]["eps_mean"] for L in Ls])
        A = np.stack([1.0 / Ls, np.ones_like(Ls)], axis=1)
        (a, b), *_ = np.linalg.lstsq(A, em, rcond=None)
        out["fit_eps_a_over_L_plus_b"] = {"a": float(a), "b": float(b)}
        T = np.array([out["per_L"][str(int(L))]["ms_per_instance_batched"] for L in Ls])
        sel = Ls >= 16
        if sel.sum() >= 2:
            out["time_alpha_batched_L_ge_16"] = float(np.polyfit(np.log(Ls[sel] ** 3), np.log(T[sel]), 1)[0])
    # App. C: eps versus beta
    plan = TnPlan(beta_L, 2, 1)
    J, egs = _batch(torch, beta_L, n_inst)
    ws = torch.empty((plan.workspace_bytes(n_inst, True) + 7) // 8, dtype=torch.float64, device="cuda")
    out["beta_study"] = {"L": beta_L, "rows": []}
    for b in betas:
        _, en, _ = tn_decimate(plan, J, b, workspace=ws, want_score=False)
        e = _eps(en, egs)
        out["beta_study"]["rows"].append({"beta": b, "eps_mean": float(e.mean()), "eps_max": float(e.max())})
        log(f"tn beta={b} L={beta_L}: eps_mean {e.mean():.5f}")
    # App. B: eps versus the fragment edge
    out["l_study"] = {"L": 20, "rows": []}
    J, egs = _batch(torch, 20, n_inst)
    for h in (1, 2):
        p = TnPlan(20, h, 1)
        w = torch.empty((p.workspace_bytes(n_inst, True) + 7) // 8, dtype=torch.float64, device="cuda")
        _, en, _ = tn_decimate(p, J, beta, workspace=w, want_score=False)
        e = _eps(en, egs)
        out["l_study"]["rows"].append({"l": 2 * h + 1, "eps_mean": float(e.mean()), "eps_max": float(e.max())})
        log(f"tn l={2 * h + 1} L=20: eps_mean {e.mean():.5f}")
    # both forms on every stand-in tile class
    out["class_study"] = {"L": 12, "rows": []}
    for h in (1, 2):
        p = TnPlan(12, h, 1)
        for cls in (-1, 0, 2, 4, 6):
            Js, egs = [], []
            for s_ in wl.tn_instances(12, n_inst):
                J, _, e = make_instance(12, cls, s_.seed)
                Js.append(np.asarray(J).reshape(6, 12 ** 3))
                egs.append(e)
            Jt = torch.from_numpy(np.stack(Js)).cuda()
            egs = np.array(egs, np.int64)
            row = {"l": 2 * h + 1, "class": cls}
            for name, (b, trop) in (("beta2", (beta, False)), ("tropical", (1.0, True))):
                _, en, _ = tn_decimate(p, Jt, b, trop, want_score=False)
                e = _eps(en, egs)
                row[name] = {"eps_mean": float(e.mean()), "eps_max": float(e.max()), "frac_exact": float(np.mean(e == 0))}
            log(f"tn class {cls} l={2 * h + 1}: {row}")
            out["class_study"]["rows"].append(row)
    return out
