// server.hip -- a continuous-batching anneal server.
//
// Requests (one replica each: an instance, a schedule, a sweep budget, a
// seed and a replica counter word) are queued by sg_server_submit.  A
// scheduler thread admits them while the device-memory budget, the active
// limit and the pool of large-lattice workspaces allow, and advances every
// active request in chunks of sweeps.  Each lattice size has its own lane
// (stream): whenever a lane's previous chunk has finished, every active
// request of that size -- including requests admitted meanwhile -- is
// launched together as the next chunk in one kernel.  A chunk continues a
// request from its absolute sweep index with the same Philox counters, so a
// request's result is identical whether it runs alone, in any mix, or in
// one piece (sa_anneal).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.hpp"
#include "variants.hpp"

using namespace sg;

namespace {

enum State : int32_t { kQueued = 0, kActive = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

double steady_now()
{
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    sg_request r;
    int32_t state = kQueued;
    int32_t done = 0;
    bool in_flight = false;
    bool cancel = false;
    double t_admit = 0.0, t_done = 0.0;
    int64_t footprint = 0;
    int ws_slot = -1;
};

struct Lane {
    int L = 0;
    const SaVariant *v = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    SaJob *h_jobs = nullptr;   // pinned staging
    SaJob *d_jobs = nullptr;
    int32_t chunk = 1;         // sweeps per chunk for this size
    bool busy = false;
    std::vector<uint64_t> chunk_ids;
    std::vector<int32_t> chunk_sweeps;
    std::vector<uint64_t> active;  // active requests of this size
};

int pick_variant(int L, const SaVariant **out)
{
    int n = 0;
    const SaVariant *vs = sa_variants(L, &n);
    if (!vs) return fail(SG_EUNSUPPORTED, "sg_server: no annealing kernel for L = %d", L);
    // one replica per request: prefer a one-replica launch shape
    for (int i = 0; i < n; ++i)
        if (vs[i].rpw == 1) {
            *out = &vs[i];
            return SG_OK;
        }
    *out = &vs[sa_selected(L)];
    return SG_OK;
}

}  // namespace

struct sg_server {
    sg_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<AdmitEntry> queue;      // arrival order
    double skip_age = 0.05;            // seconds a request may be passed over
    std::unordered_map<uint64_t, Request> reqs;
    std::map<int, std::unique_ptr<Lane>> lanes;
    std::vector<void *> ws_pool;
    std::vector<int> ws_free;
    size_t ws_bytes = 0;
    uint64_t next_id = 1;
    int64_t active = 0, mem_in_use = 0;
    sg_server_stats stats{};
    bool stop = false;
    std::string thread_error;
    std::thread th;

    ~sg_server()
    {
        for (auto &kv : lanes) {
            Lane &ln = *kv.second;
            if (ln.stream) (void)hipStreamSynchronize(ln.stream);
            if (ln.d_jobs) (void)hipFree(ln.d_jobs);
            if (ln.h_jobs) (void)hipHostFree(ln.h_jobs);
            if (ln.done) (void)hipEventDestroy(ln.done);
            if (ln.stream) (void)hipStreamDestroy(ln.stream);
        }
        for (void *p : ws_pool) (void)hipFree(p);
    }

    Lane *lane_for(int L)
    {
        auto it = lanes.find(L);
        if (it != lanes.end()) return it->second.get();
        std::unique_ptr<Lane> ln(new Lane());
        ln->L = L;
        if (pick_variant(L, &ln->v) != SG_OK) return nullptr;
        // chunks of about chunk_attempts proposals per request (at most
        // chunk_sweeps sweeps), so that chunks of all sizes take similar time
        // and no size waits long behind another in a shared hardware queue
        const int64_t N = static_cast<int64_t>(L) * L * L;
        ln->chunk = cfg.chunk_sweeps;
        if (cfg.chunk_attempts > 0)
            ln->chunk = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(cfg.chunk_sweeps,
                                                                                   cfg.chunk_attempts / N)));
        const size_t nj = static_cast<size_t>(cfg.max_active);
        if (hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln->done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&ln->h_jobs), nj * sizeof(SaJob), hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc(&ln->d_jobs, nj * sizeof(SaJob)) != hipSuccess) {
            lanes[L] = std::move(ln);  // freed by the destructor
            return nullptr;
        }
        Lane *p = ln.get();
        lanes[L] = std::move(ln);
        return p;
    }

    void release(Request &q)
    {
        mem_in_use -= q.footprint;
        if (q.ws_slot >= 0) ws_free.push_back(q.ws_slot);
        q.ws_slot = -1;
        --active;
    }

    // (lock held) retire a finished chunk of a lane
    void finish_chunk(Lane &ln)
    {
        const double t = steady_now();
        for (size_t i = 0; i < ln.chunk_ids.size(); ++i) {
            Request &q = reqs.at(ln.chunk_ids[i]);
            q.in_flight = false;
            q.done += ln.chunk_sweeps[i];
            if (q.done >= q.r.n_sweeps || q.cancel) {
                q.state = (q.done >= q.r.n_sweeps) ? kDone : kCancelled;
                q.t_done = t;
                if (q.state == kDone) {
                    ++stats.completed;
                    stats.attempts_completed += static_cast<double>(q.r.n_sweeps) * q.r.inst.L * q.r.inst.L * q.r.inst.L;
                } else {
                    ++stats.cancelled;
                }
                release(q);
                auto &act = ln.active;
                act.erase(std::remove(act.begin(), act.end(), ln.chunk_ids[i]), act.end());
            }
        }
        ln.chunk_ids.clear();
        ln.chunk_sweeps.clear();
        ln.busy = false;
    }

    // (lock held) admit queued requests that fit (admission.hpp: arrival
    // order; a request that does not fit is passed over while it is younger
    // than skip_age)
    bool admit()
    {
        AdmitCapacity cap{active, cfg.max_active, mem_in_use, cfg.memory_budget, static_cast<int64_t>(ws_free.size())};
        const double now = steady_now();
        const auto dropped = [&](uint64_t id) {
            auto it = reqs.find(id);
            return it == reqs.end() || it->second.state == kCancelled;
        };
        const std::vector<AdmitEntry> picked = admit_pick(queue, cap, now, skip_age, dropped);
        for (const AdmitEntry &e : picked) {
            Request &q = reqs.at(e.id);
            Lane *ln = lane_for(q.r.inst.L);
            if (!ln) {
                q.state = kFailed;
                q.t_done = now;
                continue;
            }
            if (e.needs_ws) {
                q.ws_slot = ws_free.back();
                ws_free.pop_back();
            }
            q.state = kActive;
            q.t_admit = now;
            mem_in_use += q.footprint;
            ++active;
            ln->active.push_back(e.id);
        }
        return !picked.empty();
    }

    // (lock held) stage the next chunk of a lane; returns the job count
    int stage(Lane &ln)
    {
        int n = 0;
        for (uint64_t id : ln.active) {
            Request &q = reqs.at(id);
            if (q.in_flight || q.state != kActive) continue;
            if (q.cancel) {  // never launched again: retire now
                q.state = kCancelled;
                q.t_done = steady_now();
                ++stats.cancelled;
                release(q);
                continue;
            }
            const int32_t chunk = std::min(ln.chunk, q.r.n_sweeps - q.done);
            SaJob &j = ln.h_jobs[n];
            std::memset(&j, 0, sizeof j);
            j.J = q.r.inst.J;
            j.jenc = q.r.inst.jenc;
            j.thr = q.r.thr + static_cast<int64_t>(q.done) * q.r.K;
            j.spins = q.r.spins;
            j.energy = q.r.energy;
            j.chain = q.r.inst.chain;
            j.rep0 = q.r.replica;
            j.n_rep = 1;
            j.n_sweeps = chunk;
            j.sweep0 = q.done;
            j.K = q.r.K;
            j.init_random = (q.done == 0) ? (q.r.init_random ? 1 : 0) : 0;
            j.k0 = static_cast<uint32_t>(q.r.seed);
            j.k1 = static_cast<uint32_t>(q.r.seed >> 32);
            j.workspace = q.ws_slot >= 0 ? static_cast<uint32_t *>(ws_pool[q.ws_slot]) : nullptr;
            q.in_flight = true;
            ln.chunk_ids.push_back(id);
            ln.chunk_sweeps.push_back(chunk);
            ++n;
        }
        // drop retired (cancelled) requests from the lane
        auto &act = ln.active;
        act.erase(std::remove_if(act.begin(), act.end(), [&](uint64_t id) { return reqs.at(id).state != kActive; }),
                  act.end());
        return n;
    }

    int launch(Lane &ln, int n)
    {
        if (hipMemcpyAsync(ln.d_jobs, ln.h_jobs, n * sizeof(SaJob), hipMemcpyHostToDevice, ln.stream) != hipSuccess)
            return fail(SG_EDEVICE, "sg_server: upload");
        const SaJob none{};
        // one replica per request: one work group per job, no group table
        const int rc = ln.v->launch(ln.d_jobs, nullptr, none, n, false, ln.stream);
        if (rc != SG_OK) return rc;
        if (hipEventRecord(ln.done, ln.stream) != hipSuccess) return fail(SG_EDEVICE, "sg_server: event");
        return SG_OK;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool progress = false;
            bool busy = false;
            for (auto &kv : lanes) {
                Lane &ln = *kv.second;
                if (ln.busy && hipEventQuery(ln.done) == hipSuccess) {
                    finish_chunk(ln);
                    progress = true;
                }
            }
            if (!stop) progress |= admit();
            for (auto &kv : lanes) {
                Lane &ln = *kv.second;
                if (ln.busy) {
                    busy = true;
                    continue;
                }
                if (ln.active.empty()) continue;
                const int n = stage(ln);
                if (n == 0) continue;
                const int rc = launch(ln, n);
                ++stats.launches;
                if (rc != SG_OK) {
                    thread_error = sg_last_error();
                    for (uint64_t id : ln.chunk_ids) {
                        Request &q = reqs.at(id);
                        q.in_flight = false;
                        q.state = kFailed;
                        q.t_done = steady_now();
                        release(q);
                    }
                    ln.chunk_ids.clear();
                    ln.chunk_sweeps.clear();
                    ln.active.clear();
                    continue;
                }
                ln.busy = true;
                busy = true;
                progress = true;
            }
            if (stop && !busy) break;
            if (progress) cv.notify_all();
            // poll the lanes' events every 50 us while work is in flight;
            // sleep until a submit otherwise
            if (busy)
                cv.wait_for(lk, std::chrono::microseconds(50));
            else if (!progress)
                cv.wait_for(lk, std::chrono::milliseconds(5));
        }
        cv.notify_all();
    }
};

extern "C" {

int sg_server_create(const sg_server_config *cfg, sg_server **out)
{
    if (!out) return fail(SG_EINVAL, "sg_server_create: NULL output");
    *out = nullptr;
    std::unique_ptr<sg_server> s(new sg_server());
    if (cfg) s->cfg = *cfg;
    if (s->cfg.max_active <= 0) s->cfg.max_active = 4096;
    if (s->cfg.chunk_sweeps <= 0) s->cfg.chunk_sweeps = 64;
    if (s->cfg.chunk_attempts < 0) return fail(SG_EINVAL, "sg_server_create: chunk_attempts < 0");
    if (s->cfg.memory_budget <= 0) s->cfg.memory_budget = int64_t(8) << 30;
    if (s->cfg.large_slots < 0) return fail(SG_EINVAL, "sg_server_create: large_slots < 0");
    if (s->cfg.skip_age_ms < 0) return fail(SG_EINVAL, "sg_server_create: skip_age_ms < 0");
    s->skip_age = (s->cfg.skip_age_ms > 0 ? s->cfg.skip_age_ms : 50) * 1e-3;
    if (hipGetDevice(&s->device) != hipSuccess) return fail(SG_EDEVICE, "sg_server_create: no device");
    s->ws_bytes = sg_sa_workspace_bytes(SG_MAX_L, 1);
    for (int i = 0; i < s->cfg.large_slots; ++i) {
        void *p = nullptr;
        if (hipMalloc(&p, s->ws_bytes) != hipSuccess) return fail(SG_ENOMEM, "sg_server_create: workspace pool");
        s->ws_pool.push_back(p);
        s->ws_free.push_back(i);
    }
    sg_server *raw = s.get();
    s->th = std::thread([raw] { raw->loop(); });
    *out = s.release();
    clear_error();
    return SG_OK;
}

double sg_server_now(const sg_server *srv)
{
    (void)srv;
    return steady_now();
}

int sg_server_submit(sg_server *srv, const sg_request *req, uint64_t *id_out)
{
    if (!srv || !req) return fail(SG_EINVAL, "sg_server_submit: NULL argument");
    const sg_instance &in = req->inst;
    if (!lattice_ok(in.L)) return fail(SG_EINVAL, "sg_server_submit: L = %d", in.L);
    int nv = 0;
    if (!sa_variants(in.L, &nv)) return fail(SG_EUNSUPPORTED, "sg_server_submit: no kernel for L = %d", in.L);
    if ((!in.J && !in.jenc) || (in.L > SG_LDS_MAX_L && !in.jenc))
        return fail(SG_EINVAL, "sg_server_submit: missing couplings (L > %d needs jenc)", SG_LDS_MAX_L);
    if (!req->thr || !req->spins || !req->energy) return fail(SG_EINVAL, "sg_server_submit: NULL array");
    if (req->n_sweeps < 1 || req->n_sweeps > (1 << 30) || req->K < 1 || req->K > SG_K_MAX)
        return fail(SG_EINVAL, "sg_server_submit: n_sweeps = %d, K = %d", req->n_sweeps, req->K);
    if ((reinterpret_cast<uintptr_t>(req->spins) & 3u) != 0)
        return fail(SG_EINVAL, "sg_server_submit: spins must be 4-byte aligned");
    const bool needs_ws = sg_sa_workspace_bytes(in.L, 1) > 0;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(SG_EBUSY, "sg_server_submit: server is shutting down");
    if (needs_ws && srv->cfg.large_slots == 0)
        return fail(SG_EUNSUPPORTED, "sg_server_submit: L = %d needs large_slots > 0", in.L);
    const uint64_t id = srv->next_id++;
    Request q;
    q.r = *req;
    q.footprint = static_cast<int64_t>(in.L) * in.L * in.L + 4 + (needs_ws ? static_cast<int64_t>(srv->ws_bytes) : 0);
    if (q.footprint > srv->cfg.memory_budget) return fail(SG_ERANGE, "sg_server_submit: request larger than the budget");
    srv->reqs.emplace(id, q);
    srv->queue.push_back(AdmitEntry{id, q.footprint, needs_ws, steady_now()});
    ++srv->stats.submitted;
    if (id_out) *id_out = id;
    srv->cv.notify_all();
    clear_error();
    return SG_OK;
}

int sg_server_poll(sg_server *srv, uint64_t id, sg_request_status *out)
{
    if (!srv || !out) return fail(SG_EINVAL, "sg_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(SG_ENOTFOUND, "sg_server_poll: unknown request %llu", (unsigned long long)id);
    const Request &q = it->second;
    out->state = q.state;
    out->done_sweeps = q.done;
    out->t_arrival = q.r.t_arrival;
    out->t_admit = q.t_admit;
    out->t_done = q.t_done;
    return SG_OK;
}

int sg_server_cancel(sg_server *srv, uint64_t id)
{
    if (!srv) return fail(SG_EINVAL, "sg_server_cancel: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(SG_ENOTFOUND, "sg_server_cancel: unknown request");
    Request &q = it->second;
    if (q.state == kQueued) {
        q.state = kCancelled;
        q.t_done = steady_now();
        ++srv->stats.cancelled;
    } else if (q.state == kActive) {
        q.cancel = true;  // retired at its next chunk boundary
    } else {
        return fail(SG_EINVAL, "sg_server_cancel: request already finished");
    }
    srv->cv.notify_all();
    return SG_OK;
}

int sg_server_release(sg_server *srv, uint64_t id)
{
    if (!srv) return fail(SG_EINVAL, "sg_server_release: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(SG_ENOTFOUND, "sg_server_release: unknown request");
    const int32_t st = it->second.state;
    if (st == kQueued || st == kActive || it->second.in_flight)
        return fail(SG_EBUSY, "sg_server_release: request %llu has not finished", (unsigned long long)id);
    srv->reqs.erase(it);
    return SG_OK;
}

int sg_server_get_stats(sg_server *srv, sg_server_stats *out)
{
    if (!srv || !out) return fail(SG_EINVAL, "sg_server_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->active = srv->active;
    out->queued = static_cast<int64_t>(srv->queue.size());
    out->memory_in_use = srv->mem_in_use;
    return SG_OK;
}

int sg_server_wait(sg_server *srv, double timeout_s)
{
    if (!srv) return fail(SG_EINVAL, "sg_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (srv->active > 0 || !srv->queue.empty()) {
        if (srv->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            std::chrono::steady_clock::now() >= deadline)
            return fail(SG_EBUSY, "sg_server_wait: timed out with %lld active, %zu queued",
                        static_cast<long long>(srv->active), srv->queue.size());
    }
    if (!srv->thread_error.empty()) return fail(SG_EDEVICE, "sg_server: %s", srv->thread_error.c_str());
    return SG_OK;
}

int sg_server_destroy(sg_server *srv)
{
    if (!srv) return SG_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (auto &kv : srv->reqs)
            if (kv.second.state == kQueued) kv.second.state = kCancelled;
            else if (kv.second.state == kActive) kv.second.cancel = true;
        srv->queue.clear();
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    delete srv;
    return SG_OK;
}

}  // extern "C"
