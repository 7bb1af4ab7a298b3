// sa.hip -- simulated annealing kernels (App. D: Metropolis sweeps over a
// beta schedule, one read = the final configuration), their launch-shape
// variants, the sa_anneal entry point and the variant autotuner.
//
// A work group anneals RPW replicas of one instance with the whole lattice
// resident in LDS: the encoded couplings once per group, RPW spin blocks,
// and the current threshold row double-buffered.  All NW*64 lanes sweep
// colour 0 units, barrier, colour 1 units, barrier.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <vector>

#include "sa_launch.hpp"

namespace sg {

// First entry of each size is its default.  RPW * L^2/2 column units per
// colour are spread over NW*64 lanes (exactly where the sizes allow).
static const SaVariant kV4[] = {SG_V(4, 16, 2, true), SG_V(4, 32, 4, true), SG_V(4, 64, 4, true),
                                SG_V(4, 64, 8, true)};
static const SaVariant kV6[] = {SG_V(6, 32, 3, true), SG_V(6, 32, 9, true), SG_V(6, 64, 9, true)};
static const SaVariant kV8[] = {SG_V(8, 16, 4, true), SG_V(8, 32, 8, true), SG_V(8, 16, 8, true),
                                SG_V(8, 1, 1, true)};
static const SaVariant kV10[] = {SG_V(10, 5, 4, true), SG_V(10, 32, 5, true), SG_V(10, 64, 10, true),
                                 SG_V(10, 32, 5, false), SG_V(10, 1, 1, true), SG_V(10, 16, 13, true)};
static const SaVariant kV12[] = {SG_V(12, 16, 9, true), SG_V(12, 16, 6, true), SG_V(12, 32, 9, true),
                                 SG_V(12, 32, 12, true), SG_V(12, 1, 1, true), SG_V(12, 8, 9, true)};
static const SaVariant kV14[] = {SG_V(14, 32, 7, false), SG_V(14, 16, 7, true), SG_V(14, 1, 2, true),
                                 SG_V(14, 10, 16, true)};
static const SaVariant kV16[] = {SG_V(16, 16, 16, true), SG_V(16, 16, 8, true), SG_V(16, 8, 8, false),
                                 SG_V(16, 8, 16, true), SG_V(16, 1, 2, true), SG_V(16, 7, 14, true),
                                 SG_V(16, 6, 12, true)};
static const SaVariant kV18[] = {SG_V(18, 8, 7, false), SG_V(18, 8, 11, false), SG_V(18, 1, 3, true),
                                 SG_V(18, 6, 16, false), SG_V(18, 6, 16, true)};
static const SaVariant kV20[] = {SG_V(20, 6, 12, true), SG_V(20, 8, 5, false), SG_V(20, 4, 5, false),
                                 SG_V(20, 1, 4, true), SG_V(20, 5, 16, false), SG_V(20, 5, 16, true)};
static const SaVariant kV22[] = {SG_V(22, 4, 8, false), SG_V(22, 4, 16, false), SG_V(22, 1, 4, true)};
static const SaVariant kV24[] = {SG_V(24, 4, 9, false), SG_V(24, 4, 6, false), SG_V(24, 1, 5, false),
                                 SG_V(24, 3, 14, false)};
// spins in LDS; couplings streamed from HBM (L2-resident), or in LDS as E
// bytes (F formed per use) of all six directions (L = 26, 28: one or two
// replicas) or of the three forward ones (more replicas, up to L = 32)
static const SaVariant kV26[] = {SG_VX(26, 2, 11, kJGlobalEF, true), SG_VX(26, 1, 6, kJGlobalEF, true),
                                 SG_VX(26, 4, 11, kJGlobalEF, true), SG_VX(26, 1, 6, kJLdsE, true),
                                 SG_VX(26, 1, 8, kJLdsE, true), SG_VX(26, 2, 11, kJLdsE, true),
                                 SG_VX(26, 2, 11, kJLds3E, true), SG_VX(26, 4, 11, kJLds3E, true)};
static const SaVariant kV28[] = {SG_VX(28, 2, 13, kJGlobalEF, true), SG_VX(28, 1, 7, kJGlobalEF, true),
                                 SG_VX(28, 4, 13, kJGlobalEF, true), SG_VX(28, 1, 7, kJLdsE, true),
                                 SG_VX(28, 1, 8, kJLdsE, true), SG_VX(28, 2, 13, kJLds3E, true),
                                 SG_VX(28, 4, 13, kJLds3E, true)};
static const SaVariant kV30[] = {SG_VX(30, 2, 15, kJGlobalEF, true), SG_VX(30, 1, 8, kJGlobalEF, true),
                                 SG_VX(30, 1, 8, kJLds3E, true), SG_VX(30, 2, 15, kJLds3E, true)};
static const SaVariant kV32[] = {SG_VX(32, 1, 8, kJLds3E, true), SG_VX(32, 2, 16, kJGlobalEF, true),
                                 SG_VX(32, 1, 8, kJGlobalEF, true)};
// couplings and spins both in HBM (a global spin workspace per replica);
// L = 34..62 are in sa_large.hip
static const SaVariant kV64[] = {SG_VX(64, 1, 16, kJGlobalEF, false), SG_VX(64, 1, 8, kJGlobalEF, false)};
#undef SG_V
#undef SG_VX

const SaVariant *sa_variants(int L, int *n)
{
#define SG_CASE(LL)                                      \
    case LL:                                             \
        *n = static_cast<int>(sizeof(kV##LL) / sizeof(kV##LL[0])); \
        return kV##LL;
    switch (L) {
        SG_CASE(4) SG_CASE(6) SG_CASE(8) SG_CASE(10) SG_CASE(12) SG_CASE(14) SG_CASE(16) SG_CASE(18)
        SG_CASE(20) SG_CASE(22) SG_CASE(24) SG_CASE(26) SG_CASE(28) SG_CASE(30) SG_CASE(32) SG_CASE(64)
    default:
        return sa_variants_large(L, n);
    }
#undef SG_CASE
}

static std::atomic<int> g_selected[SG_MAX_L + 1];

int sa_selected(int L)
{
    if (L < 0 || L > SG_MAX_L) return 0;
    return g_selected[L].load();
}

static void fill_job(SaJob &job, const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr, int8_t *spins,
                     int32_t *energy, int32_t *emin)
{
    std::memset(&job, 0, sizeof job);
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
    job.k0 = static_cast<uint32_t>(args->seed);
    job.k1 = static_cast<uint32_t>(args->seed >> 32);
    job.workspace = static_cast<uint32_t *>(args->workspace);
}

static int check_sa_args(const char *who, const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr,
                         const int8_t *spins, const int32_t *energy)
{
    if (!inst || !args) return fail(SG_EINVAL, "%s: NULL instance or args", who);
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "%s: L = %d must be even in [4, %d]", who, inst->L, SG_MAX_L);
    if (!inst->J && !inst->jenc) return fail(SG_EINVAL, "%s: instance has no couplings", who);
    if (!thr || !spins || !energy) return fail(SG_EINVAL, "%s: NULL thr, spins or energy", who);
    if (args->n_rep < 1) return fail(SG_EINVAL, "%s: n_rep = %d", who, args->n_rep);
    if (args->n_sweeps < 1) return fail(SG_EINVAL, "%s: n_sweeps = %d", who, args->n_sweeps);
    if (args->sweep0 < 0 || static_cast<int64_t>(args->sweep0) + args->n_sweeps > (1 << 30))
        return fail(SG_ERANGE, "%s: sweeps must stay below 2^30", who);
    if (args->K < 1 || args->K > SG_K_MAX) return fail(SG_EINVAL, "%s: K = %d", who, args->K);
    if (static_cast<uint64_t>(args->rep0) + static_cast<uint64_t>(args->n_rep) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "%s: replica counter words overflow", who);
    if ((reinterpret_cast<uintptr_t>(spins) & 3u) != 0) return fail(SG_EINVAL, "%s: spins must be 4-byte aligned", who);
    int nv = 0;
    if (!sa_variants(inst->L, &nv)) return fail(SG_EUNSUPPORTED, "%s: no annealing kernel for L = %d", who, inst->L);
    if (inst->L > SG_LDS_MAX_L && !inst->jenc)
        return fail(SG_EINVAL, "%s: L = %d needs the encoded couplings (sg_encode_instance)", who, inst->L);
    const size_t ws = sg_sa_workspace_bytes(inst->L, args->n_rep);
    if (ws > 0) {
        if (!args->workspace || args->workspace_bytes < static_cast<int64_t>(ws))
            return fail(SG_EINVAL, "%s: L = %d needs a %zu-byte workspace", who, inst->L, ws);
        if ((reinterpret_cast<uintptr_t>(args->workspace) & 15u) != 0)
            return fail(SG_EINVAL, "%s: workspace must be 16-byte aligned", who);
    }
    return SG_OK;
}

int sa_check_job(const sg_sa_job &j, int index)
{
    char who[64];
    std::snprintf(who, sizeof who, "sg_batch_create: job %d", index);
    return check_sa_args(who, &j.inst, &j.args, j.thr, j.spins, j.energy);
}

void sa_fill_job(SaJob &job, const sg_sa_job &j)
{
    fill_job(job, &j.inst, &j.args, j.thr, j.spins, j.energy, j.emin);
}

// sa_anneal's own choice of the multi-work-group path: the selected
// single-work-group kernel would launch too few groups to fill the device
static bool wide_auto(int L, int n_rep)
{
    int n = 0;
    const SaVariant *vs = sa_variants(L, &n);
    if (!vs || n_rep < 1 || !wide_supported(L)) return false;
    const int rpw = vs[sa_selected(L)].rpw;
    return (n_rep + rpw - 1) / rpw < SG_WIDE_MAX_GROUPS;
}

static int run_variant(const SaVariant &v, const SaJob &job, hipStream_t st)
{
    const int groups = (job.n_rep + v.rpw - 1) / v.rpw;
    return v.launch(nullptr, nullptr, job, groups, job.emin != nullptr, st);
}

}  // namespace sg

using namespace sg;

extern "C" {

int sa_anneal(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr, int8_t *spins, int32_t *energy,
              int32_t *emin, void *stream)
{
    const int rc = check_sa_args("sa_anneal", inst, args, thr, spins, energy);
    if (rc != SG_OK) return rc;
    int n = 0;
    const SaVariant *vs = sa_variants(inst->L, &n);
    if (!vs) return fail(SG_EUNSUPPORTED, "sa_anneal: L = %d", inst->L);
    SaJob job;
    fill_job(job, inst, args, thr, spins, energy, emin);
    clear_error();
    // few replicas of a large lattice: spread over the device
    const int L = inst->L;
    if (!emin && wide_auto(L, args->n_rep) && args->workspace &&
        (reinterpret_cast<uintptr_t>(args->workspace) & 15u) == 0 &&
        args->workspace_bytes >= static_cast<int64_t>(wide_bytes(L, args->n_rep)))
        return sa_wide(job, L, static_cast<hipStream_t>(stream));
    return run_variant(vs[sa_selected(inst->L)], job, static_cast<hipStream_t>(stream));
}

int sg_sa_anneal_wide(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr, int8_t *spins,
                      int32_t *energy, void *stream)
{
    const int rc = check_sa_args("sg_sa_anneal_wide", inst, args, thr, spins, energy);
    if (rc != SG_OK) return rc;
    if (!wide_supported(inst->L))
        return fail(SG_EUNSUPPORTED, "sg_sa_anneal_wide: L = %d (the wide path covers even L = 26..64)", inst->L);
    const size_t need = wide_bytes(inst->L, args->n_rep);
    if (!args->workspace || args->workspace_bytes < static_cast<int64_t>(need))
        return fail(SG_EINVAL, "sg_sa_anneal_wide: needs a %zu-byte workspace", need);
    if ((reinterpret_cast<uintptr_t>(args->workspace) & 15u) != 0)
        return fail(SG_EINVAL, "sg_sa_anneal_wide: workspace must be 16-byte aligned");
    SaJob job;
    fill_job(job, inst, args, thr, spins, energy, nullptr);
    clear_error();
    return sa_wide(job, inst->L, static_cast<hipStream_t>(stream));
}

size_t sg_sa_wide_workspace_bytes(int32_t L, int32_t n_rep)
{
    return wide_auto(L, n_rep) ? wide_bytes(L, n_rep) : 0;
}

int sg_sa_variants(int32_t L, int32_t max, sg_sa_variant *out)
{
    int n = 0;
    const SaVariant *vs = sa_variants(L, &n);
    if (!vs) return fail(SG_EUNSUPPORTED, "sg_sa_variants: L = %d has no LDS-resident variants", L);
    for (int i = 0; i < n && i < max && out; ++i) {
        out[i].L = vs[i].L;
        out[i].replicas_per_group = vs[i].rpw;
        out[i].waves_per_group = vs[i].nw;
        out[i].both_encodings = vs[i].jf;
        out[i].couplings_in_hbm = vs[i].jglobal;
        out[i].spins_in_hbm = vs[i].sglobal;
        out[i].lds_bytes = static_cast<int64_t>(vs[i].lds_bytes);
    }
    return n;
}

size_t sg_sa_workspace_bytes(int32_t L, int32_t n_rep)
{
    if (!lattice_ok(L) || n_rep < 1 || L <= 32) return 0;
    const size_t H = L / 2, NC = H * L, C = (L + 3) / 4;
    return static_cast<size_t>(n_rep) * 2 * NC * C * sizeof(uint32_t);
}

int sg_sa_select_variant(int32_t L, int32_t variant)
{
    int n = 0;
    if (!sa_variants(L, &n)) return fail(SG_EUNSUPPORTED, "sg_sa_select_variant: L = %d", L);
    if (variant < 0 || variant >= n) return fail(SG_EINVAL, "sg_sa_select_variant: variant %d of %d", variant, n);
    g_selected[L].store(variant);
    return SG_OK;
}

int sg_sa_selected_variant(int32_t L)
{
    int n = 0;
    if (!sa_variants(L, &n)) return fail(SG_EUNSUPPORTED, "sg_sa_selected_variant: L = %d", L);
    return sa_selected(L);
}

int sg_sa_anneal_variant(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr, int8_t *spins,
                         int32_t *energy, int32_t *emin, int32_t variant, void *stream)
{
    const int rc = check_sa_args("sg_sa_anneal_variant", inst, args, thr, spins, energy);
    if (rc != SG_OK) return rc;
    int n = 0;
    const SaVariant *vs = sa_variants(inst->L, &n);
    if (variant < 0 || variant >= n) return fail(SG_EINVAL, "sg_sa_anneal_variant: variant %d of %d", variant, n);
    SaJob job;
    fill_job(job, inst, args, thr, spins, energy, emin);
    clear_error();
    return run_variant(vs[variant], job, static_cast<hipStream_t>(stream));
}

}  // extern "C"
