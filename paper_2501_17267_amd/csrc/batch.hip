// batch.hip -- batched simulated annealing: many jobs of different L in one
// schedule, one kernel per L on parallel graph branches.
#include <algorithm>
#include <map>
#include <memory>
#include <vector>

#include "common.hpp"
#include "sa_kernel.hpp"

namespace sg {

struct Group {
    int32_t job;    // index into the bucket's job table
    int32_t group;  // replica group inside the job
};

template <int L, int RPW, int NW, bool JF, bool TRACK>
__global__ __launch_bounds__(NW * 64) void k_sa_batch(const SaJob *jobs, const Group *groups)
{
    const Group g = groups[blockIdx.x];
    const SaJob job = jobs[g.job];
    sa_group<L, RPW, NW, JF, TRACK>(job, g.group, job.k0, job.k1);
}

template <int L>
static int launch_bucket(const SaJob *d_jobs, const Group *d_groups, int n_groups, bool track, hipStream_t st)
{
    using Cfg = SaCfg<L>;
    (void)hipGetLastError();  // clear a stale error so the check below sees this launch only
    if (track)
        hipLaunchKernelGGL((k_sa_batch<L, Cfg::RPW, Cfg::NW, Cfg::JF, true>), dim3(n_groups), dim3(Cfg::NW * 64), 0,
                           st, d_jobs, d_groups);
    else
        hipLaunchKernelGGL((k_sa_batch<L, Cfg::RPW, Cfg::NW, Cfg::JF, false>), dim3(n_groups), dim3(Cfg::NW * 64),
                           0, st, d_jobs, d_groups);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_batch_launch: %s", hipGetErrorString(err));
    return SG_OK;
}

static int replicas_per_group(int L)
{
    switch (L) {
#define SG_RPW(LL) \
    case LL: return SaCfg<LL>::RPW;
        SG_RPW(4) SG_RPW(6) SG_RPW(8) SG_RPW(10) SG_RPW(12) SG_RPW(14) SG_RPW(16) SG_RPW(18) SG_RPW(20)
        SG_RPW(22) SG_RPW(24)
#undef SG_RPW
    default: return 0;
    }
}

static int launch_bucket_any(int L, const SaJob *j, const Group *g, int n, bool track, hipStream_t st)
{
    switch (L) {
#define SG_BK(LL) \
    case LL: return launch_bucket<LL>(j, g, n, track, st);
        SG_BK(4) SG_BK(6) SG_BK(8) SG_BK(10) SG_BK(12) SG_BK(14) SG_BK(16) SG_BK(18) SG_BK(20) SG_BK(22)
        SG_BK(24)
#undef SG_BK
    default: return fail(SG_EUNSUPPORTED, "sg_batch: L = %d", L);
    }
}

}  // namespace sg

using namespace sg;

struct sg_batch {
    struct Bucket {
        int L = 0;
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
            const int rc = launch_bucket_any(b.L, b.d_jobs, b.d_groups, b.n_groups, b.track, b.stream);
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
        const sg_sa_job &j = jobs[i];
        const int L = j.inst.L;
        if (!lattice_ok(L) || L > SG_LDS_MAX_L) return fail(SG_EUNSUPPORTED, "sg_batch_create: job %d has L = %d", i, L);
        if ((!j.inst.J && !j.inst.jenc) || !j.thr || !j.spins || !j.energy)
            return fail(SG_EINVAL, "sg_batch_create: job %d has a NULL array", i);
        if (j.args.n_rep < 1 || j.args.n_sweeps < 1 || j.args.K < 1 || j.args.K > SG_K_MAX || j.args.sweep0 < 0 ||
            static_cast<int64_t>(j.args.sweep0) + j.args.n_sweeps > (1 << 30))
            return fail(SG_EINVAL, "sg_batch_create: job %d has invalid arguments", i);
        if (static_cast<uint64_t>(j.args.rep0) + static_cast<uint64_t>(j.args.n_rep) > 0xFFFFFFFFull)
            return fail(SG_ERANGE, "sg_batch_create: job %d replica words overflow", i);
        if ((reinterpret_cast<uintptr_t>(j.spins) & 3u) != 0)
            return fail(SG_EINVAL, "sg_batch_create: job %d spins not 4-byte aligned", i);
        by_L[L].push_back(i);
    }
    std::unique_ptr<sg_batch> b(new sg_batch());
    b->use_graph = (flags & SG_BATCH_GRAPH) != 0;
    if (hipGetDevice(&b->device) != hipSuccess) return fail(SG_EDEVICE, "sg_batch_create: no device");
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return fail(SG_EDEVICE, "sg_batch_create: event");
    for (auto &kv : by_L) {
        const int L = kv.first;
        const int rpw = replicas_per_group(L);
        sg_batch::Bucket bk;
        bk.L = L;
        std::vector<SaJob> hj;
        std::vector<Group> hg;
        for (int idx : kv.second) {
            const sg_sa_job &j = jobs[idx];
            SaJob s{};
            s.J = j.inst.J;
            s.jenc = j.inst.jenc;
            s.thr = j.thr;
            s.spins = j.spins;
            s.energy = j.energy;
            s.emin = j.emin;
            s.chain = j.inst.chain;
            s.rep0 = j.args.rep0;
            s.n_rep = j.args.n_rep;
            s.n_sweeps = j.args.n_sweeps;
            s.sweep0 = j.args.sweep0;
            s.K = j.args.K;
            s.init_random = j.args.init_random ? 1 : 0;
            s.k0 = static_cast<uint32_t>(j.args.seed);
            s.k1 = static_cast<uint32_t>(j.args.seed >> 32);
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
