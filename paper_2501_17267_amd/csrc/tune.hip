// tune.hip -- autotuner of the simulated-annealing launch shapes.
//
// For one lattice size it anneals the same synthetic instance with every
// compiled variant (replicas per work group, waves per work group, coupling
// encoding), requires bit-identical spins and energies from all of them
// (the chain depends only on its Philox counters, never on the launch
// shape), times each with device events, and selects the fastest for every
// later sa_anneal call and batch plan of that size.
#include <algorithm>
#include <cstring>
#include <vector>

#include "variants.hpp"

using namespace sg;

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t n) { return hipMalloc(&p, n) == hipSuccess; }
};

}  // namespace

extern "C" int sg_autotune_sa(int32_t L, int32_t n_rep, int32_t n_sweeps, int32_t repeats, sg_sa_tune_result *out,
                              int32_t max_out, void *stream)
{
    int nv = 0;
    const SaVariant *vs = sa_variants(L, &nv);
    if (!vs) return fail(SG_EUNSUPPORTED, "sg_autotune_sa: L = %d has no LDS-resident variants", L);
    if (n_rep < 1 || n_sweeps < 1 || repeats < 1) return fail(SG_EINVAL, "sg_autotune_sa: bad sizes");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t N = static_cast<int64_t>(L) * L * L;
    std::vector<int8_t> J(6 * N), planted(N);
    int64_t egs = 0;
    int rc = sg_make_instance(L, 6, 0x7E57ull + static_cast<uint64_t>(L), J.data(), planted.data(), &egs);
    if (rc != SG_OK) return rc;
    std::vector<double> beta(n_sweeps);
    rc = sg_make_schedule(0, 0.1, 3.0, n_sweeps, beta.data());
    if (rc != SG_OK) return rc;
    std::vector<uint32_t> thr(static_cast<size_t>(n_sweeps) * SG_K_MAX);
    rc = sg_make_thresholds(beta.data(), n_sweeps, SG_K_MAX, thr.data());
    if (rc != SG_OK) return rc;

    DevBuf dJ, dThr, dSpins, dE, dJenc, dWs;
    const size_t spin_bytes = static_cast<size_t>(n_rep) * N;
    const size_t ws_bytes = sg_sa_workspace_bytes(L, n_rep);
    if (!dJ.alloc(J.size()) || !dThr.alloc(thr.size() * 4) || !dSpins.alloc(spin_bytes * nv) ||
        !dE.alloc(static_cast<size_t>(n_rep) * 4 * nv) || !dJenc.alloc(sg_jenc_bytes(L)) ||
        (ws_bytes > 0 && !dWs.alloc(ws_bytes)))
        return fail(SG_ENOMEM, "sg_autotune_sa: device allocation");
    if (hipMemcpy(dJ.p, J.data(), J.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dThr.p, thr.data(), thr.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(SG_EDEVICE, "sg_autotune_sa: upload");

    sg_instance inst{};
    inst.L = L;
    inst.J = static_cast<const int8_t *>(dJ.p);
    inst.E_gs = egs;
    inst.chain = 0x5EED;
    if (L > SG_LDS_MAX_L) {
        rc = sg_encode_instance(&inst, static_cast<uint32_t *>(dJenc.p), st);
        if (rc != SG_OK) return rc;
        inst.jenc = static_cast<const uint32_t *>(dJenc.p);
    }
    sg_sa_args args{};
    args.n_rep = n_rep;
    args.n_sweeps = n_sweeps;
    args.K = SG_K_MAX;
    args.init_random = 1;
    args.seed = 0x0DDBA11ull;
    args.workspace = dWs.p;
    args.workspace_bytes = static_cast<int64_t>(ws_bytes);

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SG_EDEVICE, "sg_autotune_sa: events");
    std::vector<float> ms(nv, 0.0f);
    int status = SG_OK;
    for (int v = 0; v < nv && status == SG_OK; ++v) {
        int8_t *sp = static_cast<int8_t *>(dSpins.p) + spin_bytes * v;
        int32_t *en = static_cast<int32_t *>(dE.p) + static_cast<size_t>(n_rep) * v;
        status = sg_sa_anneal_variant(&inst, &args, static_cast<const uint32_t *>(dThr.p), sp, en, nullptr, v, st);
        if (status != SG_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < repeats && status == SG_OK; ++r)
            status = sg_sa_anneal_variant(&inst, &args, static_cast<const uint32_t *>(dThr.p), sp, en, nullptr, v, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) status = fail(SG_EDEVICE, "sg_autotune_sa: synchronize");
        if (status == SG_OK && hipEventElapsedTime(&ms[v], e0, e1) != hipSuccess)
            status = fail(SG_EDEVICE, "sg_autotune_sa: timing");
        ms[v] /= static_cast<float>(repeats);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != SG_OK) return status;

    // every variant must reproduce variant 0 bit for bit
    std::vector<int8_t> ref(spin_bytes), got(spin_bytes);
    std::vector<int32_t> eref(n_rep), egot(n_rep);
    if (hipMemcpy(ref.data(), dSpins.p, spin_bytes, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(eref.data(), dE.p, static_cast<size_t>(n_rep) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(SG_EDEVICE, "sg_autotune_sa: download");
    std::vector<int> identical(nv, 1);
    for (int v = 1; v < nv; ++v) {
        if (hipMemcpy(got.data(), static_cast<int8_t *>(dSpins.p) + spin_bytes * v, spin_bytes,
                      hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(egot.data(), static_cast<int32_t *>(dE.p) + static_cast<size_t>(n_rep) * v,
                      static_cast<size_t>(n_rep) * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(SG_EDEVICE, "sg_autotune_sa: download");
        identical[v] = (got == ref) && (egot == eref);
    }
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (identical[v] && ms[v] < ms[best]) best = v;
    for (int v = 0; v < nv && out && v < max_out; ++v) {
        out[v].variant = v;
        out[v].ms = ms[v];
        out[v].attempts_per_s = static_cast<double>(n_rep) * n_sweeps * static_cast<double>(N) / (ms[v] * 1e-3);
        out[v].identical = identical[v];
    }
    for (int v = 1; v < nv; ++v)
        if (!identical[v]) return fail(SG_EDEVICE, "sg_autotune_sa: variant %d of L = %d differs from variant 0", v, L);
    const int sel = sg_sa_select_variant(L, best);
    if (sel != SG_OK) return sel;
    clear_error();
    return best;
}
