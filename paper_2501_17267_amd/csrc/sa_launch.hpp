// sa_launch.hpp -- the simulated-annealing kernel entry and the launch of
// one variant (replicas per group, waves per group, coupling placement,
// spin placement), shared by the translation units that instantiate the
// variants of each lattice size.
#pragma once

#include "variants.hpp"

namespace sg {

template <int L, int RPW, int NW, int JM, bool SL, bool TRACK>
__global__ __launch_bounds__(NW * 64) void k_sa(const SaJob *jobs, const Group *groups, SaJob inline_job)
{
    if (jobs == nullptr) {
        sa_group<L, RPW, NW, JM, SL, TRACK>(inline_job, static_cast<int>(blockIdx.x), inline_job.k0, inline_job.k1);
    } else {
        // groups == NULL: one group per job, job index = block index
        const Group g = groups ? groups[blockIdx.x] : Group{static_cast<int32_t>(blockIdx.x), 0};
        const SaJob job = jobs[g.job];
        sa_group<L, RPW, NW, JM, SL, TRACK>(job, g.group, job.k0, job.k1);
    }
}

template <int L, int RPW, int NW, int JM, bool SL>
static int launch_variant(const SaJob *jobs, const Group *groups, const SaJob &inline_job, int n_groups, bool track,
                          hipStream_t stream)
{
    (void)hipGetLastError();  // clear a stale error so the check below sees this launch only
    if (track)
        hipLaunchKernelGGL((k_sa<L, RPW, NW, JM, SL, true>), dim3(n_groups), dim3(NW * 64), 0, stream, jobs, groups,
                           inline_job);
    else
        hipLaunchKernelGGL((k_sa<L, RPW, NW, JM, SL, false>), dim3(n_groups), dim3(NW * 64), 0, stream, jobs, groups,
                           inline_job);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "annealing kernel launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

template <int L, int JM, bool SL>
constexpr size_t lds_of(int rpw)
{
    using G = Geo<L>;
    const int jdw = (JM == kJGlobalEF) ? 0 : (JM == kJLdsE ? G::JDW_E : (JM == kJLds3E ? G::JDW_3E : G::JDW_EF));
    return 4 * (((2 * kThrEntries + 3 * rpw + 3) & ~3) + jdw + (SL ? rpw * G::SPIN_DW : 0));
}

#define SG_VX(L, RPW, NW, JM, SL) \
    {L, RPW, NW, ((JM) == kJLdsE || (JM) == kJLds3E) ? 0 : 1, (JM) == kJGlobalEF ? 1 : 0, SL ? 0 : 1, lds_of<L, JM, SL>(RPW), \
     &launch_variant<L, RPW, NW, JM, SL>}
#define SG_V(L, RPW, NW, JF) SG_VX(L, RPW, NW, (JF) ? kJLdsEF : kJLdsE, true)

}  // namespace sg
