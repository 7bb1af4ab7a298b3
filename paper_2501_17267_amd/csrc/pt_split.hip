// pt_split.hip -- sg_pt_run_split: parallel tempering (App. D) with each
// run spread over G work groups (the kernel and its mailbox protocol are in
// pt.hpp).  For fewer runs than compute units: the one-group form leaves
// the rest of the device idle.
#include <mutex>

#include "pt.hpp"

namespace sg {

constexpr size_t kPtSplitHeader = 256;   // status word, padded
constexpr int kPtSplitMinUnits = 512;
constexpr int64_t kPtSplitMinSites = 6144;

}  // namespace sg

using namespace sg;

extern "C" size_t sg_pt_split_workspace_bytes(int32_t n_runs, int32_t T)
{
    if (n_runs < 1 || T < 2 || T > SG_PT_MAX_T) return 0;
    return kPtSplitHeader + static_cast<size_t>(n_runs) * 2 * static_cast<size_t>(T) * sizeof(uint64_t);
}

namespace sg {

// The split launch on a given workspace (mailbox after a kPtSplitHeader
// header).  status: where the give-up flag goes (NULL: the header's first
// int32).
static int pt_split_impl(const char *who, const sg_instance *inst, const sg_pt_args *args, int32_t groups,
                         int32_t waves, const uint32_t *thr, const uint32_t *thrx, int8_t *spins, int32_t *energy_out,
                         int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc, void *workspace,
                         int64_t workspace_bytes, int32_t *status, void *stream)
{
    PtJob job;
    const int rc = pt_prepare(inst, args, thr, thrx, spins, energy_out, pos, emin_trace, swap_acc, who, job);
    if (rc != SG_OK) return rc;
    if (groups != 0 && groups != 1 && groups != 2 && groups != 4 && groups != 8)
        return fail(SG_EINVAL, "%s: groups = %d must be 0, 1, 2, 4 or 8", who, groups);
    if (groups > 0 && args->T % groups != 0)
        return fail(SG_EINVAL, "%s: T = %d is not a multiple of groups = %d", who, args->T, groups);
    if (waves != 0 && waves != 4 && waves != 8 && waves != 12 && waves != 16)
        return fail(SG_EINVAL, "%s: waves = %d must be 0, 4, 8, 12 or 16", who, waves);
    if (groups == 0) {
        // the most groups per run (dividing T) whose launch has at most one
        // work group per compute unit.  When one group per run would already
        // keep at least half the device busy, every group must also keep at
        // least kPtSplitMinUnits column units per colour (below that the
        // per-step exchange of energies outweighs the smaller sweep).  With
        // fewer runs the idle compute units decide, and the split pays even
        // with small groups (one run: 1.3 to 2.9 times faster per step)
        // unless a run's whole step is already below the split form's
        // floor of about 2.4 us (T * N under kPtSplitMinSites).
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return fail(SG_EDEVICE, "%s: device query failed", who);
        const int64_t chunks = (static_cast<int64_t>(args->n_runs) + 7) / 8;
        const int64_t sites = static_cast<int64_t>(args->T) * inst->L * inst->L * inst->L;
        const bool few_runs = 2 * static_cast<int64_t>(args->n_runs) < n_cu && sites >= kPtSplitMinSites;
        groups = 1;
        for (int gg : {2, 4, 8})
            if (args->T % gg == 0 && chunks * 8 * gg <= n_cu &&
                (few_runs || args->T / gg * inst->L * inst->L / 2 >= kPtSplitMinUnits))
                groups = gg;
    }
    const uint32_t k0 = static_cast<uint32_t>(args->seed), k1 = static_cast<uint32_t>(args->seed >> 32);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t need = sg_pt_split_workspace_bytes(args->n_runs, args->T);
    if (groups > 1 || workspace) {
        if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 7u) != 0)
            return fail(SG_EINVAL, "%s: workspace must be a non-NULL 8-byte aligned device pointer", who);
        if (workspace_bytes < 0 || static_cast<size_t>(workspace_bytes) < need)
            return fail(SG_EINVAL, "%s: workspace of %lld bytes, %zu needed", who,
                        static_cast<long long>(workspace_bytes), need);
    }
    job.status = status ? status : static_cast<int32_t *>(workspace);
    job.mbox = workspace ? reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + kPtSplitHeader) : nullptr;
    clear_error();
    // the launcher clears the mailbox (split form) and the status word on the
    // stream, after its own checks, just before the PT kernel
    if (groups == 1) return pt_dispatch<false>(inst->L, job, args->n_runs, waves ? waves : pt_waves(inst->L, args->T),
                                               k0, k1, st, who);
    job.G = groups;
    const int nw = waves ? waves : pt_split_waves(args->T / groups * inst->L * inst->L / 2);
    return pt_dispatch<true>(inst->L, job, args->n_runs, nw, k0, k1, st, who);
}

// No-allocation form: the workspace is a fixed device array of this
// translation unit.  In host code `scratch` names a host-side stand-in, not
// device memory; its device address (one copy per GPU) comes from
// hipGetSymbolAddress on the first call on each device and is kept.
constexpr size_t kPtStaticScratchBytes = SG_PT_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) uint64_t scratch[kPtStaticScratchBytes / sizeof(uint64_t)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int static_scratch(const char *who, void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SG_EDEVICE, "%s: no current device", who);
    if (dev < 0 || dev >= kMaxDevices) return fail(SG_EUNSUPPORTED, "%s: device %d beyond %d", who, dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p)
            return fail(SG_EDEVICE, "%s: address of the static workspace: %s", who, hipGetErrorString(err));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SG_OK;
}

}  // namespace sg

extern "C" int sg_pt_run_split(const sg_instance *inst, const sg_pt_args *args, int32_t groups, int32_t waves,
                               const uint32_t *thr, const uint32_t *thrx, int8_t *spins, int32_t *energy_out,
                               int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc, void *workspace,
                               int64_t workspace_bytes, void *stream)
{
    return pt_split_impl("sg_pt_run_split", inst, args, groups, waves, thr, thrx, spins, energy_out, pos, emin_trace,
                         swap_acc, workspace, workspace_bytes, nullptr, stream);
}

extern "C" int sg_pt_run_split_static(const sg_instance *inst, const sg_pt_args *args, int32_t groups,
                                      int32_t waves, const uint32_t *thr, const uint32_t *thrx, int8_t *spins,
                                      int32_t *energy_out, int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc,
                                      int32_t *status_out, void *stream)
{
    const char *who = "sg_pt_run_split_static";
    if (!args) return fail(SG_EINVAL, "%s: NULL args", who);
    const size_t need = sg_pt_split_workspace_bytes(args->n_runs, args->T);
    if (need == 0) return fail(SG_EINVAL, "%s: n_runs = %d, T = %d", who, args->n_runs, args->T);
    if (need > kPtStaticScratchBytes)
        return fail(SG_ERANGE, "%s: %d runs of %d walkers need %zu bytes of workspace, above the static %zu",
                    who, args->n_runs, args->T, need, kPtStaticScratchBytes);
    if (status_out && (reinterpret_cast<uintptr_t>(status_out) & 3u) != 0)
        return fail(SG_EINVAL, "%s: status_out must be 4-byte aligned", who);
    void *ws = nullptr;
    const int rc = static_scratch(who, &ws);
    if (rc != SG_OK) return rc;
    return pt_split_impl(who, inst, args, groups, waves, thr, thrx, spins, energy_out, pos, emin_trace, swap_acc, ws,
                         static_cast<int64_t>(kPtStaticScratchBytes), status_out, stream);
}
