// batch.hip -- batched simulated annealing: many jobs of different L in one
// schedule, one kernel per L on parallel graph branches.
#include <algorithm>
#include <map>
#include <memory>
#include <vector>

#include "common.hpp"
#include "variants.hpp"

namespace sg {

int sa_check_job(const sg_sa_job &j, int index);
void sa_fill_job(SaJob &job, const sg_sa_job &j);

}  // namespace sg

using namespace sg;

struct sg_batch {
    struct Bucket {
        int L = 0;
        int variant = 0;
        const SaVariant *v = nullptr;
        bool track = false;
        int n_groups = 0;
        SaJob *d_jobs = nullptr;
        Group *d_groups = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        hipEvent_t t0 = nullptr, t1 = nullptr;  // kernel start / end of the last launch
        double attempts = 0.0;
    };
    std::vector<Bucket> buckets;
    int64_t n_groups = 0;
    double attempts = 0.0;
    hipEvent_t fork = nullptr;
    bool use_graph = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t capture = nullptr;
    int device = 0;

    ~sg_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto &b : buckets) {
            if (b.d_jobs) (void)hipFree(b.d_jobs);
            if (b.d_groups) (void)hipFree(b.d_groups);
            if (b.done) (void)hipEventDestroy(b.done);
            if (b.t0) (void)hipEventDestroy(b.t0);
            if (b.t1) (void)hipEventDestroy(b.t1);
            if (b.stream) (void)hipStreamDestroy(b.stream);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (capture) (void)hipStreamDestroy(capture);
    }

    // fork onto the bucket streams, launch, join back into `st`
    bool timed = false;  // the last launch recorded kernel timing events

    int enqueue(hipStream_t st, bool capturing)
    {
        if (hipEventRecord(fork, st) != hipSuccess) return fail(SG_EDEVICE, "sg_batch: event record");
        for (auto &b : buckets) {
            if (hipStreamWaitEvent(b.stream, fork, 0) != hipSuccess) return fail(SG_EDEVICE, "sg_batch: wait");
            // kernel timing events only outside graph capture (timing events
            // recorded inside a captured graph cannot be queried)
            if (!capturing && hipEventRecord(b.t0, b.stream) != hipSuccess)
                return fail(SG_EDEVICE, "sg_batch: event record");
            const SaJob none{};
            const int rc = b.v->launch(b.d_jobs, b.d_groups, none, b.n_groups, b.track, b.stream);
            if (rc != SG_OK) return rc;
            if (!capturing && hipEventRecord(b.t1, b.stream) != hipSuccess)
                return fail(SG_EDEVICE, "sg_batch: event record");
            if (hipEventRecord(b.done, b.stream) != hipSuccess) return fail(SG_EDEVICE, "sg_batch: event record");
            if (hipStreamWaitEvent(st, b.done, 0) != hipSuccess) return fail(SG_EDEVICE, "sg_batch: join");
        }
        return SG_OK;
    }
};

extern "C" {

int sg_batch_create(const sg_sa_job *jobs, int32_t n_jobs, int32_t flags, sg_batch **out)
{
    if (!jobs || n_jobs < 1 || !out) return fail(SG_EINVAL, "sg_batch_create: no jobs");
    *out = nullptr;
    std::map<int, std::vector<int>> by_L;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const int rc = sa_check_job(jobs[i], i);
        if (rc != SG_OK) return rc;
        by_L[jobs[i].inst.L].push_back(i);
    }
    std::unique_ptr<sg_batch> b(new sg_batch());
    b->use_graph = (flags & SG_BATCH_GRAPH) != 0;
    if (hipGetDevice(&b->device) != hipSuccess) return fail(SG_EDEVICE, "sg_batch_create: no device");
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return fail(SG_EDEVICE, "sg_batch_create: event");
    for (auto &kv : by_L) {
        const int L = kv.first;
        int nv = 0;
        const SaVariant *vs = sa_variants(L, &nv);
        if (!vs) return fail(SG_EUNSUPPORTED, "sg_batch_create: L = %d", L);
        sg_batch::Bucket bk;
        bk.L = L;
        bk.variant = sa_selected(L);
        bk.v = &vs[bk.variant];
        const int rpw = bk.v->rpw;
        std::vector<SaJob> hj;
        std::vector<Group> hg;
        for (int idx : kv.second) {
            const sg_sa_job &j = jobs[idx];
            SaJob s;
            sa_fill_job(s, j);
            if (j.emin) bk.track = true;
            const int g_count = (s.n_rep + rpw - 1) / rpw;
            for (int g = 0; g < g_count; ++g) hg.push_back(Group{static_cast<int32_t>(hj.size()), g});
            const double att = static_cast<double>(s.n_rep) * s.n_sweeps * static_cast<double>(L) * L * L;
            b->attempts += att;
            bk.attempts += att;
            hj.push_back(s);
        }
        // longest work first, so the hardware dispatcher fills the tail with short groups
        std::stable_sort(hg.begin(), hg.end(), [&](const Group &a, const Group &c) {
            return hj[a.job].n_sweeps > hj[c.job].n_sweeps;
        });
        bk.n_groups = static_cast<int>(hg.size());
        b->n_groups += bk.n_groups;
        if (hipMalloc(&bk.d_jobs, hj.size() * sizeof(SaJob)) != hipSuccess ||
            hipMalloc(&bk.d_groups, hg.size() * sizeof(Group)) != hipSuccess) {
            b->buckets.push_back(bk);
            return fail(SG_ENOMEM, "sg_batch_create: device allocation");
        }
        b->buckets.push_back(bk);
        auto &last = b->buckets.back();
        if (hipMemcpy(last.d_jobs, hj.data(), hj.size() * sizeof(SaJob), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(last.d_groups, hg.data(), hg.size() * sizeof(Group), hipMemcpyHostToDevice) != hipSuccess)
            return fail(SG_EDEVICE, "sg_batch_create: upload");
        if (hipStreamCreateWithFlags(&last.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&last.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&last.t0) != hipSuccess || hipEventCreate(&last.t1) != hipSuccess)
            return fail(SG_EDEVICE, "sg_batch_create: stream");
    }
    if (b->use_graph) {
        if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
            return fail(SG_EDEVICE, "sg_batch_create: capture stream");
        if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(SG_EDEVICE, "sg_batch_create: begin capture");
        const int rc = b->enqueue(b->capture, true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (rc != SG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(SG_EDEVICE, "sg_batch_create: end capture: %s", hipGetErrorString(e));
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
            return fail(SG_EDEVICE, "sg_batch_create: instantiate");
    }
    *out = b.release();
    clear_error();
    return SG_OK;
}

int sg_batch_launch(sg_batch *b, void *stream)
{
    if (!b) return fail(SG_EINVAL, "sg_batch_launch: NULL plan");
    hipStream_t st = static_cast<hipStream_t>(stream);
    clear_error();
    if (b->use_graph) {
        const hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return fail(SG_EDEVICE, "sg_batch_launch: %s", hipGetErrorString(e));
        b->timed = false;
        return SG_OK;
    }
    const int rc = b->enqueue(st, false);
    b->timed = (rc == SG_OK);
    return rc;
}

int sg_batch_info(const sg_batch *b, int32_t *n_kernels, int64_t *n_groups, double *attempts)
{
    if (!b) return fail(SG_EINVAL, "sg_batch_info: NULL plan");
    if (n_kernels) *n_kernels = static_cast<int32_t>(b->buckets.size());
    if (n_groups) *n_groups = b->n_groups;
    if (attempts) *attempts = b->attempts;
    return SG_OK;
}

int sg_batch_kernels(const sg_batch *b, int32_t n, int32_t *L_out, double *attempts_out, float *ms_out)
{
    if (!b) return fail(SG_EINVAL, "sg_batch_kernels: NULL plan");
    const int32_t m = std::min<int32_t>(n, static_cast<int32_t>(b->buckets.size()));
    for (int32_t i = 0; i < m; ++i) {
        const auto &bk = b->buckets[i];
        if (L_out) L_out[i] = bk.L;
        if (attempts_out) attempts_out[i] = bk.attempts;
        if (ms_out) {
            float ms = -1.0f;
            if (!b->timed || hipEventElapsedTime(&ms, bk.t0, bk.t1) != hipSuccess) {
                ms = -1.0f;
                (void)hipGetLastError();  // do not leave a stale error for the next call
            }
            ms_out[i] = ms;
        }
    }
    return m;
}

int sg_batch_destroy(sg_batch *b)
{
    if (!b) return SG_OK;
    (void)hipSetDevice(b->device);
    for (auto &bk : b->buckets)
        if (bk.stream) (void)hipStreamSynchronize(bk.stream);
    if (b->capture) (void)hipStreamSynchronize(b->capture);
    (void)hipDeviceSynchronize();
    delete b;
    return SG_OK;
}

}  // extern "C"
