// variants.hpp -- launch shapes of the simulated-annealing kernel.
//
// A variant fixes, for one lattice size L, the replicas per work group
// (RPW), the waves per work group (NW) and whether LDS holds both coupling
// encodings (E and F) or E only.  They trade LDS per group (occupancy)
// against VALU work per site; the autotuner times them on the device.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "sa_kernel.hpp"

namespace sg {

// jobs == NULL: one job passed by value (inline_job), group = blockIdx.x
using SaLaunchFn = int (*)(const SaJob *jobs, const Group *groups, const SaJob &inline_job, int n_groups,
                           bool track, hipStream_t stream);

struct SaVariant {
    int L, rpw, nw, jf, jglobal, sglobal;
    size_t lds_bytes;
    SaLaunchFn launch;
};

// variants of lattice size L (count written to *n); NULL when L has none
const SaVariant *sa_variants(int L, int *n);
// variants of the sizes between L = 32 and 64 (sa_large.hip)
const SaVariant *sa_variants_large(int L, int *n);
// currently selected variant index of L (default or autotuned)
int sa_selected(int L);

// energies (Eq. 1) of n configurations in natural order (aux.hip)
int launch_energy(const int8_t *J, int L, int n, const int8_t *spins, int32_t *out, hipStream_t stream);

// multi-work-group anneal of lattices above the LDS-resident sizes
// (wide.hip): sizes it covers, the workspace it needs, and the launch
bool wide_supported(int L);
size_t wide_bytes(int L, int n_rep);
int sa_wide(const SaJob &job, int L, hipStream_t stream);

}  // namespace sg
