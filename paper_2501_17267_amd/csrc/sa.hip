// sa.hip -- simulated annealing kernel (App. D: Metropolis sweeps over a beta
// schedule, one read = the final configuration) and its C-ABI entry point.
//
// A work group anneals RPW replicas of one instance with the whole lattice
// resident in LDS: the encoded couplings once per group, RPW spin blocks,
// and the current threshold row double-buffered.  All NW*64 lanes sweep
// colour 0 units, barrier, colour 1 units, barrier.
#include <algorithm>

#include "common.hpp"
#include "sa_kernel.hpp"

namespace sg {

template <int L, int RPW, int NW, bool JF, bool TRACK>
__global__ __launch_bounds__(NW * 64) void k_sa(SaJob job, uint32_t k0, uint32_t k1)
{
    sa_group<L, RPW, NW, JF, TRACK>(job, static_cast<int>(blockIdx.x), k0, k1);
}

template <int L, int RPW, int NW, bool JF>
static int launch_sa(const SaJob &job, uint32_t k0, uint32_t k1, hipStream_t stream)
{
    const int groups = (job.n_rep + RPW - 1) / RPW;
    (void)hipGetLastError();  // clear a stale error so the check below sees this launch only
    if (job.emin)
        hipLaunchKernelGGL((k_sa<L, RPW, NW, JF, true>), dim3(groups), dim3(NW * 64), 0, stream, job, k0, k1);
    else
        hipLaunchKernelGGL((k_sa<L, RPW, NW, JF, false>), dim3(groups), dim3(NW * 64), 0, stream, job, k0, k1);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sa_anneal: launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

int dispatch_sa(int L, const SaJob &job, uint32_t k0, uint32_t k1, hipStream_t stream)
{
    switch (L) {
#define SG_SA_CASE(LL)                                                                  \
    case LL:                                                                            \
        return launch_sa<LL, SaCfg<LL>::RPW, SaCfg<LL>::NW, SaCfg<LL>::JF>(job, k0, k1, \
                                                                           stream);
        SG_SA_CASE(4)
        SG_SA_CASE(6)
        SG_SA_CASE(8)
        SG_SA_CASE(10)
        SG_SA_CASE(12)
        SG_SA_CASE(14)
        SG_SA_CASE(16)
        SG_SA_CASE(18)
        SG_SA_CASE(20)
        SG_SA_CASE(22)
        SG_SA_CASE(24)
#undef SG_SA_CASE
    default:
        return fail(SG_EUNSUPPORTED, "sa_anneal: L = %d needs the streaming kernel", L);
    }
}

}  // namespace sg

using namespace sg;

extern "C" int sa_anneal(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr,
                         int8_t *spins, int32_t *energy, int32_t *emin, void *stream)
{
    if (!inst || !args) return fail(SG_EINVAL, "sa_anneal: NULL instance or args");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "sa_anneal: L = %d must be even in [4, %d]", inst->L, SG_MAX_L);
    if (!inst->J && !inst->jenc) return fail(SG_EINVAL, "sa_anneal: instance has no couplings");
    if (!thr || !spins || !energy) return fail(SG_EINVAL, "sa_anneal: NULL thr, spins or energy");
    if (args->n_rep < 1) return fail(SG_EINVAL, "sa_anneal: n_rep = %d", args->n_rep);
    if (args->n_sweeps < 1) return fail(SG_EINVAL, "sa_anneal: n_sweeps = %d", args->n_sweeps);
    if (args->sweep0 < 0 || static_cast<int64_t>(args->sweep0) + args->n_sweeps > (1 << 30))
        return fail(SG_ERANGE, "sa_anneal: sweeps must stay below 2^30");
    if (args->K < 1 || args->K > SG_K_MAX) return fail(SG_EINVAL, "sa_anneal: K = %d", args->K);
    if (static_cast<uint64_t>(args->rep0) + static_cast<uint64_t>(args->n_rep) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "sa_anneal: replica counter words overflow");
    if ((reinterpret_cast<uintptr_t>(spins) & 3u) != 0)
        return fail(SG_EINVAL, "sa_anneal: spins must be 4-byte aligned");
    if (inst->L > SG_LDS_MAX_L) return fail(SG_EUNSUPPORTED, "sa_anneal: L = %d above the LDS-resident range", inst->L);
    SaJob job{};
    job.J = inst->J;
    job.jenc = inst->jenc;
    job.thr = thr;
    job.spins = spins;
    job.energy = energy;
    job.emin = emin;
    job.chain = inst->chain;
    job.rep0 = args->rep0;
    job.n_rep = args->n_rep;
    job.n_sweeps = args->n_sweeps;
    job.sweep0 = args->sweep0;
    job.K = args->K;
    job.init_random = args->init_random ? 1 : 0;
    clear_error();
    return dispatch_sa(inst->L, job, static_cast<uint32_t>(args->seed),
                       static_cast<uint32_t>(args->seed >> 32), static_cast<hipStream_t>(stream));
}
