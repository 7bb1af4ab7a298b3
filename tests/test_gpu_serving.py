"""The anneal server: every request's result equals one sa_anneal call of
the same request, whether it is served alone or in a mix, whatever the
chunk size, the admission limits or the other requests; cancellation and
budget-limited admission behave."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from paper_2501_17267_amd import serving
from paper_2501_17267_amd import workloads as wl
from gpu_util import dev_u32, log

pytestmark = pytest.mark.gpu
SEED = 0x5EB7


def _setup(sizes=(8, 12, 16, 20, 26, 32, 64), n=36, seed=11):
    rng = np.random.default_rng(seed)
    insts = {L: sg.Instance.generate(L, 1000 + L, chain=L) for L in sizes}
    reqs = []
    for i in range(n):
        L = int(sizes[i % len(sizes)])
        S = int(rng.integers(3, 40)) if L < 64 else int(rng.integers(2, 9))
        thr = dev_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, S)))
        reqs.append({"L": L, "S": S, "thr": thr, "replica": 100 + i})
    return insts, reqs


def _serve(srv, insts, reqs, order=None):
    out = []
    for i in (order or range(len(reqs))):
        r = reqs[i]
        sp = torch.empty(r["L"] ** 3, dtype=torch.int8, device="cuda")
        en = torch.empty(1, dtype=torch.int32, device="cuda")
        rid = srv.submit(insts[r["L"]], r["thr"], SEED, r["replica"], sp, en)
        out.append((i, rid, sp, en))
    srv.wait(120)
    return out


def _alone_call(insts, r):
    sp, en, _ = sg.sa_anneal(insts[r["L"]], r["thr"], 1, SEED, rep0=r["replica"])
    torch.cuda.synchronize()
    return sp[0], en[0]


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_served_results_equal_single_calls(chunk):
    log(f"serving chunk={chunk}")
    insts, reqs = _setup()
    srv = serving.Server(max_active=64, chunk_sweeps=chunk, large_slots=4)
    got = _serve(srv, insts, reqs)
    for i, rid, sp, en in got:
        st = srv.poll(rid)
        assert st["state"] == serving.SG_REQ_DONE and st["done_sweeps"] == reqs[i]["S"]
        a_sp, a_en = _alone_call(insts, reqs[i])
        assert torch.equal(sp, a_sp), (i, reqs[i]["L"])
        assert int(en[0]) == int(a_en)
    stats = srv.stats()
    assert stats["completed"] == len(reqs) and stats["active"] == 0 and stats["memory_in_use"] == 0
    srv.close()


def test_alone_equals_in_mix_and_tight_admission():
    insts, reqs = _setup(n=24, seed=5)
    # in a mix with everything admitted at once
    srv = serving.Server(max_active=1024, chunk_sweeps=5, large_slots=8)
    mix = {i: (sp.clone(), en.clone()) for i, rid, sp, en in _serve(srv, insts, reqs, order=list(range(24))[::-1])}
    srv.close()
    # one at a time: a budget that admits a single small request
    srv = serving.Server(max_active=1, chunk_sweeps=3, memory_budget=600000, large_slots=1)
    for i, rid, sp, en in _serve(srv, insts, reqs):
        assert torch.equal(sp, mix[i][0]) and torch.equal(en, mix[i][1]), i
    srv.close()


def test_cancel_queued_and_active():
    insts, reqs = _setup(sizes=(16,), n=6, seed=3)
    long_thr = dev_u32(sg.make_thresholds(sg.make_schedule(0, 0.1, 3.0, 4000)))
    srv = serving.Server(max_active=1, chunk_sweeps=16, large_slots=0)
    sp = [torch.empty(16 ** 3, dtype=torch.int8, device="cuda") for _ in range(3)]
    en = [torch.empty(1, dtype=torch.int32, device="cuda") for _ in range(3)]
    a = srv.submit(insts[16], long_thr, SEED, 1, sp[0], en[0])
    b = srv.submit(insts[16], long_thr, SEED, 2, sp[1], en[1])
    srv.cancel(b)   # still queued behind a (max_active = 1)
    srv.cancel(a)   # active: retired at its next chunk boundary
    c = srv.submit(insts[16], reqs[0]["thr"], SEED, 3, sp[2], en[2])
    srv.wait(60)
    assert srv.poll(a)["state"] == serving.SG_REQ_CANCELLED
    assert srv.poll(b)["state"] == serving.SG_REQ_CANCELLED
    assert srv.poll(c)["state"] == serving.SG_REQ_DONE
    a_sp, a_en = _alone_call(insts, {"L": 16, "thr": reqs[0]["thr"], "replica": 3})
    assert torch.equal(sp[2], a_sp)
    with pytest.raises(sg.SgError):
        srv.poll(987654)
    srv.close()


def test_short_poisson_stream():
    res = serving.run_poisson(torch, rate=400.0, duration=2.0, warmup=0.5, pool=2, chunk=32,
                              plain_sample=8, check_sample=8, log=log)
    log(f"short stream: {res}")
    assert res["served_equals_alone"]
    assert res["completed_all"] == res["submitted"]


def test_served_stream_sample_against_oracle():
    # a short stream with the serving workload's mix (L even 8..32 and 5 %
    # L = 64, sweeps log-uniform 64..4096, one replica per request): served
    # requests whose chains the oracle finishes in about a second each are
    # re-run on the oracle from their own instance, schedule and counters
    def inst_seed(L, k):
        return wl.mix64(0xABC000 + 131 * L + k)
    res = serving.run_poisson(torch, rate=400.0, duration=2.0, warmup=0.0, pool=2, chunk=64,
                              plain_sample=2, check_sample=2, log=log, p_large=0.05,
                              instance_seed=inst_seed, return_requests=True)
    d = res.pop("requests_detail")
    st, off, N = d["stream"], d["off"], d["N"]
    cost = N * st["S"]
    order = np.argsort(cost, kind="stable")
    small = [int(i) for i in order if st["L"][i] != 64 and cost[i] <= 2e7][:10]
    large = [int(i) for i in order if st["L"][i] == 64 and cost[i] <= 4e7][:1]
    sample = small + large
    log(f"served-vs-oracle sample: {[(int(st['L'][i]), int(st['S'][i])) for i in sample]}")
    assert len(small) >= 5
    en = d["energy"].cpu().numpy()
    for i in sample:
        L, k, S = int(st["L"][i]), int(st["k"][i]), int(st["S"][i])
        inst = d["insts"][(L, k)]
        Jo, _, egs = oracle.make_instance(L, 6, inst_seed(L, k))
        assert egs == inst.E_gs
        thr_h = oracle.thresholds(oracle.schedule(0, 0.1, 3.0, S), 24)
        sp_ref, e_ref, _ = oracle.sa_run(L, Jo, d["key"], inst.chain, thr_h, n_rep=1, rep0=i)
        got = d["spins"][int(off[i]):int(off[i]) + int(N[i])].cpu().numpy()
        np.testing.assert_array_equal(got, sp_ref[0], err_msg=f"request {i} L={L} S={S}")
        assert int(en[i]) == int(e_ref[0]), i
