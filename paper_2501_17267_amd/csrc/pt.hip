// pt.hip -- pt_run: parallel tempering (App. D), one work group per run
// (the kernel is in pt.hpp).
#include "pt.hpp"

using namespace sg;

extern "C" int pt_run(const sg_instance *inst, const sg_pt_args *args, const uint32_t *thr,
                      const uint32_t *thrx, int8_t *spins, int32_t *energy_out, int32_t *pos,
                      int32_t *emin_trace, uint32_t *swap_acc, void *stream)
{
    PtJob job;
    const int rc = pt_prepare(inst, args, thr, thrx, spins, energy_out, pos, emin_trace, swap_acc, "pt_run", job);
    if (rc != SG_OK) return rc;
    clear_error();
    const uint32_t k0 = static_cast<uint32_t>(args->seed), k1 = static_cast<uint32_t>(args->seed >> 32);
    return pt_dispatch<false>(inst->L, job, args->n_runs, pt_waves(inst->L, args->T), k0, k1,
                              static_cast<hipStream_t>(stream), "pt_run");
}
