// pt.hip -- parallel tempering kernel (App. D) and its C-ABI entry point.
//
// One work group runs one PT run: the T walkers of the run, the encoded
// couplings and the T rows of thresholds are LDS-resident.  A step is a
// colour-0 pass over all walkers' columns, a colour-1 pass, then the
// even/odd replica exchange done by one lane per ladder pair, all inside
// the group, so a run never leaves its compute unit.
#include <algorithm>

#include "common.hpp"
#include "sweep.hpp"

namespace sg {

struct PtJob {
    const int8_t *J;
    const uint32_t *jenc;
    const uint32_t *thr;    // [T][K]
    const uint32_t *thrx;   // [T-1][M]
    int8_t *spins;          // [n_runs][T][N]
    int32_t *energy;        // [n_runs][T]
    int32_t *pos;           // [n_runs][T]
    int32_t *emin_trace;    // [n_runs][n_steps] or NULL
    uint32_t *swap_acc;     // [n_runs][T-1] or NULL
    uint32_t run0;
    int32_t T;
    int32_t n_steps;
    int32_t step0;
    int32_t K;
    int32_t M;
    int32_t init_random;
    int32_t mx;             // exchange-table entries per ladder pair copied to LDS
};

constexpr int kPtThr = kThrEntries;  // table entries per ladder slot

template <int L>
struct PtCfg {
    static constexpr bool JF = (L <= 12);
};

// Waves per work group for T walkers of size L: the T * L^2/2 column units
// of a colour phase are dealt to NW * 64 lanes in ceil(units / (NW*64))
// passes.  Pick the NW with the least idle lane-passes (passes * NW), the
// larger NW on ties (more waves to hide LDS latency).
constexpr int kPtWaves[] = {4, 8, 12, 16};
inline int pt_waves(int L, int T)
{
    const int units = T * L * L / 2;
    int best = 4, best_cost = 1 << 30;
    for (int nw : kPtWaves) {
        const int passes = (units + nw * 64 - 1) / (nw * 64);
        const int cost = passes * nw;
        if (cost < best_cost || (cost == best_cost && nw > best)) {
            best = nw;
            best_cost = cost;
        }
    }
    return best;
}

// LDS of one run: T spin blocks, the couplings, T threshold tables, four
// per-walker words and the first mx entries of each pair's exchange table
template <int L, bool JF>
constexpr size_t pt_lds_bytes(int T, int mx)
{
    using G = Geo<L>;
    return (static_cast<size_t>(T) * G::SPIN_DW + (JF ? G::JDW_EF : G::JDW_E) +
            static_cast<size_t>(T) * kPtThr + 4 * static_cast<size_t>(T) +
            static_cast<size_t>(T - 1) * static_cast<size_t>(mx)) * 4;
}

// Units (walker, column) a lane may hold prepared (neighbours and the
// sweep-independent Philox products, as in the annealing kernel): the
// register file gives each lane 512 / ceil(NW/4) registers, about 100 of
// which the sweep itself needs; a prepared unit takes 4 per dword + 8.
template <int L, int NW>
constexpr int pt_umax()
{
    constexpr int regs = 512 / ((NW + 3) / 4) - 100;
    constexpr int per = 4 * Geo<L>::C + 8;
    return (regs / per) < 4 ? regs / per : 4;
}

template <int L, int NW, bool JF, bool PREP>
__global__ __launch_bounds__(NW * 64) void k_pt(PtJob job, uint32_t k0, uint32_t k1)
{
    using G = Geo<L>;
    using Col = Column<L, JF>;
    constexpr int NT = NW * 64;
    constexpr int JDW = JF ? G::JDW_EF : G::JDW_E;
    extern __shared__ uint32_t lds[];
    const int T = job.T;
    uint32_t *s_spin = lds;
    uint32_t *s_j = s_spin + T * G::SPIN_DW;
    uint32_t *s_thr = s_j + JDW;
    int32_t *s_E = reinterpret_cast<int32_t *>(s_thr + T * kPtThr);
    int32_t *s_pos = s_E + T;
    int32_t *s_who = s_pos + T;
    int32_t *s_sw = s_who + T;
    uint32_t *s_thrx = reinterpret_cast<uint32_t *>(s_sw + T);
    const int mx = job.mx;

    const int tid = static_cast<int>(threadIdx.x);
    const int run = static_cast<int>(blockIdx.x);
    const uint32_t chain = job.run0 + static_cast<uint32_t>(run);
    int8_t *spins = job.spins + static_cast<int64_t>(run) * T * G::N;

    // ---- set-up ---------------------------------------------------------
    for (int w = tid; w < T * G::SPIN_DW; w += NT) s_spin[w] = 0u;
    for (int w = tid; w < T * kPtThr; w += NT) {
        const int slot = w / kPtThr, e = w - slot * kPtThr;
        s_thr[w] = thr_entry(job.thr + slot * job.K, job.K, e);
    }
    for (int w = tid; w < (T - 1) * mx; w += NT) {
        const int k = w / mx, e = w - k * mx;
        s_thrx[w] = job.thrx[static_cast<int64_t>(k) * job.M + e];
    }
    if (tid < T) {
        s_E[tid] = 0;
        s_sw[tid] = 0;
        int p = job.init_random ? tid : job.pos[run * T + tid];
        if (p < 0 || p >= T) p = tid;  // keeps LDS indices in range; pos must be a permutation
        s_pos[tid] = p;
    }
    load_couplings<L, JF>(s_j, job.J, job.jenc, tid, NT);
    __syncthreads();
    if (tid < T) s_who[s_pos[tid]] = tid;
    {
        uint8_t *sb = reinterpret_cast<uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < T * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            load_spins_one<L>(sb + wk * G::SPIN_DW * 4, q, job.init_random != 0,
                              spins + static_cast<int64_t>(wk) * G::N, static_cast<uint32_t>(wk), chain,
                              k0, k1);
        }
    }
    __syncthreads();
    for (int u = tid; u < T * G::NC; u += NT) {
        const int wk = u / G::NC;
        const int col = u - wk * G::NC;
        atomicAdd(&s_E[wk], Col::column_energy_of(s_spin + wk * G::SPIN_DW, s_j, col));
    }
    __syncthreads();

    // prepared units: a lane keeps the same (walker, column) units for the
    // whole run (the launcher guarantees they number at most UMAX)
    constexpr int UMAX = PREP ? pt_umax<L, NW>() : 1;
    typename Col::Unit un[UMAX];
    int wks[UMAX];
    bool act[UMAX];
    if constexpr (PREP) {
#pragma unroll
        for (int i = 0; i < UMAX; ++i) {
            const int u = tid + i * NT;
            act[i] = u < T * G::NC;
            const int ua = act[i] ? u : 0;
            const int wk = ua / G::NC;
            wks[i] = wk;
            un[i] = Col::make_unit(ua - wk * G::NC, static_cast<uint32_t>(wk), chain, k0, k1);
        }
    }

    // ---- steps ------------------------------------------------------------
    for (int ti = 0; ti < job.n_steps; ++ti) {
        const uint32_t t = static_cast<uint32_t>(job.step0 + ti);
        if constexpr (PREP) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int i = 0; i < UMAX; ++i) {
                    if (!act[i]) continue;
                    const int wk = wks[i];
                    const int32_t dE = Col::template metropolis_unit<true>(
                        s_spin + wk * G::SPIN_DW, s_j, s_thr + s_pos[wk] * kPtThr, c, un[i],
                        2u * t + static_cast<uint32_t>(c), k0, k1);
                    if (dE != 0) atomicAdd(&s_E[wk], dE);
                }
                __syncthreads();
            }
        } else {
            for (int c = 0; c < 2; ++c) {
                for (int u = tid; u < T * G::NC; u += NT) {
                    const int wk = u / G::NC;
                    const int col = u - wk * G::NC;
                    const int32_t dE = Col::template metropolis<true>(
                        s_spin + wk * G::SPIN_DW, s_j, s_thr + s_pos[wk] * kPtThr, c, col,
                        2u * t + static_cast<uint32_t>(c), static_cast<uint32_t>(wk), chain, k0, k1);
                    if (dE != 0) atomicAdd(&s_E[wk], dE);
                }
                __syncthreads();
            }
        }
        // exchange of ladder pairs (k, k+1), k = t mod 2, t mod 2 + 2, ...
        const int k = tid;
        if (k + 1 < T && ((k ^ static_cast<int>(t)) & 1) == 0) {
            const int a = s_who[k], b = s_who[k + 1];
            const int32_t D = s_E[a] - s_E[b];
            bool acc = D <= 0;
            if (!acc) {
                const int32_t m = D / 2;
                const Rand4 u = philox10(static_cast<uint32_t>(k), t, 0xFFFFFFFFu, chain, k0, k1);
                if (m <= mx)
                    acc = u.w[0] < s_thrx[k * mx + (m - 1)];
                else
                    acc = (m <= job.M) && (u.w[0] < job.thrx[static_cast<int64_t>(k) * job.M + (m - 1)]);
            }
            if (acc) {
                s_who[k] = b;
                s_who[k + 1] = a;
                s_pos[b] = k;
                s_pos[a] = k + 1;
                s_sw[k] += 1;
            }
        }
        if (job.emin_trace && tid >= 64 && tid < 128) {
            const int lane = tid - 64;
            int32_t e = 0x7FFFFFFF;
            for (int w = lane; w < T; w += 64) e = min(e, s_E[w]);
            for (int off = 32; off > 0; off >>= 1) e = min(e, __shfl_xor(e, off, 64));
            if (lane == 0) job.emin_trace[static_cast<int64_t>(run) * job.n_steps + ti] = e;
        }
        __syncthreads();
    }

    // ---- write-back ---------------------------------------------------------
    {
        const uint8_t *sb = reinterpret_cast<const uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < T * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            store_spins_one<L>(sb + wk * G::SPIN_DW * 4, q, spins + static_cast<int64_t>(wk) * G::N);
        }
    }
    if (tid < T) {
        job.energy[run * T + tid] = s_E[tid];
        job.pos[run * T + tid] = s_pos[tid];
        if (job.swap_acc && tid + 1 < T) job.swap_acc[run * (T - 1) + tid] += static_cast<uint32_t>(s_sw[tid]);
    }
}

template <int L, int NW>
static int launch_pt_nw(PtJob job, int n_runs, uint32_t k0, uint32_t k1, hipStream_t stream)
{
    using Cfg = PtCfg<L>;
    constexpr size_t kLds = 160 * 1024;
    const size_t base = pt_lds_bytes<L, Cfg::JF>(job.T, 0);
    if (base > kLds)
        return fail(SG_EUNSUPPORTED, "pt_run: L = %d with T = %d needs %zu bytes of LDS", L, job.T, base);
    // the exchange-table prefix held in LDS: up to 128 entries per pair,
    // as many as the LDS left over allows (later entries are read from HBM)
    job.mx = static_cast<int32_t>(std::min<size_t>({static_cast<size_t>(job.M), 128,
                                                   (kLds - base) / (4 * static_cast<size_t>(job.T - 1))}));
    const size_t bytes = pt_lds_bytes<L, Cfg::JF>(job.T, job.mx);
    const int units = job.T * Geo<L>::NC;
    const int upl = (units + NW * 64 - 1) / (NW * 64);
    auto kern = (upl <= pt_umax<L, NW>()) ? k_pt<L, NW, Cfg::JF, true> : k_pt<L, NW, Cfg::JF, false>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (err != hipSuccess) return fail(SG_EDEVICE, "pt_run: LDS attribute: %s", hipGetErrorString(err));
    (void)hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(n_runs), dim3(NW * 64), bytes, stream, job, k0, k1);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "pt_run: launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

template <int L>
static int launch_pt(const PtJob &job, int n_runs, uint32_t k0, uint32_t k1, hipStream_t stream)
{
    switch (pt_waves(L, job.T)) {
    case 4: return launch_pt_nw<L, 4>(job, n_runs, k0, k1, stream);
    case 8: return launch_pt_nw<L, 8>(job, n_runs, k0, k1, stream);
    case 12: return launch_pt_nw<L, 12>(job, n_runs, k0, k1, stream);
    default: return launch_pt_nw<L, 16>(job, n_runs, k0, k1, stream);
    }
}

}  // namespace sg

using namespace sg;

extern "C" int pt_run(const sg_instance *inst, const sg_pt_args *args, const uint32_t *thr,
                      const uint32_t *thrx, int8_t *spins, int32_t *energy_out, int32_t *pos,
                      int32_t *emin_trace, uint32_t *swap_acc, void *stream)
{
    if (!inst || !args) return fail(SG_EINVAL, "pt_run: NULL instance or args");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "pt_run: L = %d must be even in [4, %d]", inst->L, SG_MAX_L);
    if (!inst->J && !inst->jenc) return fail(SG_EINVAL, "pt_run: instance has no couplings");
    if (!thr || !thrx || !spins || !energy_out || !pos) return fail(SG_EINVAL, "pt_run: NULL array");
    if (args->n_runs < 1 || args->n_steps < 1) return fail(SG_EINVAL, "pt_run: n_runs = %d, n_steps = %d", args->n_runs, args->n_steps);
    if (args->T < 2 || args->T > SG_PT_MAX_T) return fail(SG_EINVAL, "pt_run: T = %d outside [2, %d]", args->T, SG_PT_MAX_T);
    if (args->K < 1 || args->K > SG_K_MAX || args->M < 1) return fail(SG_EINVAL, "pt_run: K = %d, M = %d", args->K, args->M);
    if (args->step0 < 0 || static_cast<int64_t>(args->step0) + args->n_steps > (1 << 30))
        return fail(SG_ERANGE, "pt_run: steps must stay below 2^30");
    if (static_cast<uint64_t>(args->run0) + static_cast<uint64_t>(args->n_runs) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "pt_run: run counter words overflow");
    if ((reinterpret_cast<uintptr_t>(spins) & 3u) != 0) return fail(SG_EINVAL, "pt_run: spins must be 4-byte aligned");
    PtJob job{};
    job.J = inst->J;
    job.jenc = inst->jenc;
    job.thr = thr;
    job.thrx = thrx;
    job.spins = spins;
    job.energy = energy_out;
    job.pos = pos;
    job.emin_trace = emin_trace;
    job.swap_acc = swap_acc;
    job.run0 = args->run0;
    job.T = args->T;
    job.n_steps = args->n_steps;
    job.step0 = args->step0;
    job.K = args->K;
    job.M = args->M;
    job.init_random = args->init_random ? 1 : 0;
    clear_error();
    const uint32_t k0 = static_cast<uint32_t>(args->seed), k1 = static_cast<uint32_t>(args->seed >> 32);
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (inst->L) {
    case 4: return launch_pt<4>(job, args->n_runs, k0, k1, st);
    case 6: return launch_pt<6>(job, args->n_runs, k0, k1, st);
    case 8: return launch_pt<8>(job, args->n_runs, k0, k1, st);
    case 10: return launch_pt<10>(job, args->n_runs, k0, k1, st);
    case 12: return launch_pt<12>(job, args->n_runs, k0, k1, st);
    case 14: return launch_pt<14>(job, args->n_runs, k0, k1, st);
    case 16: return launch_pt<16>(job, args->n_runs, k0, k1, st);
    default: return fail(SG_EUNSUPPORTED, "pt_run: L = %d is above the LDS-resident PT range", inst->L);
    }
}
