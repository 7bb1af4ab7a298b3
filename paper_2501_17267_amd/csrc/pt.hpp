// pt.hpp -- the parallel tempering kernel (App. D), shared by the
// one-group-per-run entry point (pt.hip) and the split form (pt_split.hip).
//
// One work group holds the walkers it sweeps, the encoded couplings and the
// T rows of thresholds in LDS.  A step is a colour-0 pass over its walkers'
// columns, a colour-1 pass, then the even/odd replica exchange done by one
// lane per ladder pair.
//
// Without SPLIT a work group runs a whole PT run, so a run never leaves its
// compute unit.  With SPLIT a run's T walkers are dealt to G work groups
// (T/G each, walker w in group w / (T/G)); after each step's sweep every
// group publishes its walkers' energies as 64-bit words (step tag in the
// high half, energy in the low half) in a device-memory mailbox and reads
// the other groups' words of the same step.  Every group then holds all T
// energies and makes the same exchange decisions from the same Philox
// counters, so the ladder stays identical in every group and the results
// are those of the one-group kernel, bit for bit.
//
// Mailbox safety: step ti writes half (ti mod 2) of the run's mailbox with
// tag ti + 1.  A group overwrites that half again only at step ti + 2,
// after its exchange of step ti + 1, which needs every other group's tag
// ti + 2 word, which each group writes only after reading the tag ti + 1
// words.  So no word is overwritten before every group has read it, and a
// reader never sees a later tag than the one it waits for.  The mailbox is
// zeroed by a fill kernel queued before the PT kernel (tags start at 1).
#pragma once

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
    int32_t n_runs;
    int32_t G;              // work groups per run (SPLIT)
    uint64_t *mbox;         // [n_runs][2][T] tagged energies (SPLIT)
    int32_t *status;        // bit 0: a wait on another group gave up (SPLIT); bit 1: pos was no permutation
};

constexpr int kPtThr = kThrEntries;  // table entries per ladder slot

// A wait for another group's energies polls at most this many times (each
// poll is a device-scope load of about a microsecond, then a short sleep);
// past that the run is abandoned: status is set, later waits are skipped
// and the kernel still runs to its end.
constexpr int kPtPollLimit = 1 << 22;

// Couplings in LDS as E = J + 8 only (F = 8 - J formed in registers): the
// sweep's LDS reads, not its VALU work, bound the PT step, and storing both
// halves doubles the coupling reads (measured at L = 8 and 12: E only runs
// the PT workloads 1.3 to 1.4 times faster).  They use the odd-stride
// arrangement (kColMajorOdd).
template <int L>
struct PtCfg {
    static constexpr bool JF = false;
};

// Waves per work group for `units` column units of a colour phase dealt to
// NW * 64 lanes in ceil(units / (NW*64)) passes.  Pick the NW with the
// least idle lane-passes (passes * NW), the larger NW on ties (more waves
// to hide LDS latency).
constexpr int kPtWaves[] = {4, 8, 12, 16};
inline int pt_waves_for_units(int units)
{
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

inline int pt_waves(int L, int T) { return pt_waves_for_units(T * L * L / 2); }

// Waves per work group of the split form, whose groups mostly have a compute
// unit each: the fewest passes, then the fewest waves that reach them.
inline int pt_split_waves(int units)
{
    int best = 4, best_passes = 1 << 30;
    for (int nw : kPtWaves) {
        const int passes = (units + nw * 64 - 1) / (nw * 64);
        if (passes < best_passes) {
            best = nw;
            best_passes = passes;
        }
    }
    return best;
}

// LDS of one work group: its spin blocks (TG walkers), the couplings, T
// threshold tables, four per-walker words and the first mx entries of each
// pair's exchange table
template <int L, bool JF>
constexpr size_t pt_lds_bytes(int TG, int T, int mx)
{
    using G = Geo<L>;
    return (static_cast<size_t>(TG) * G::SPIN_DW + G::jdw_odd(JF ? 2 : 1) +
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

// Prepared units per lane whose colour-0 random words of the coming step
// are drawn while wave 0 trades energies with the other groups (split form)
// or runs the exchange (one group per run); the words follow from the
// Philox counter alone, not from the ladder position the exchange settles.
// Each holds 4 registers per dword until the sweep.  Counts read off the
// gfx950 register allocation for L = 4..16: two units at 12 waves (one at
// L = 16) and three at 8 spill nothing and keep the work groups a compute
// unit holds; at 16 waves no register is free, and at 4 the extra
// registers cost L = 10 and 12 a resident work group.
template <int L, int NW, int UMAX>
constexpr int pt_npre()
{
    constexpr int n = NW == 12 ? (L >= 16 ? 1 : 2) : NW == 8 ? 3 : 0;
    return n < UMAX ? n : UMAX;
}

// One Metropolis pass over colour 0 of a prepared unit with random words
// drawn beforehand: the result of Column::metropolis_unit for c = 0.
template <int L, class Col>
__device__ __forceinline__ int32_t pt_colour0_drawn(uint32_t *rep, const uint32_t *jl, const uint32_t *thr,
                                                    const typename Col::Unit &un, const Rand4 (&u)[Col::C])
{
    int32_t dE = 0;
    uint32_t own[Col::C], kb[Col::C];
    Col::fields_n(rep, jl, 0, un.n.self, un.n, own, kb);
    const char *tb = reinterpret_cast<const char *>(thr);
#pragma unroll
    for (int m = 0; m < Col::C; ++m) own[m] ^= Col::template accept_dword<true>(kb[m], u[m], tb, m, dE);
#pragma unroll
    for (int m = 0; m < Col::C; ++m) rep[spin_at<L, kColMajor>(0, un.n.self, m)] = own[m];
    return dE;
}

// UMAX: prepared units per lane (0: units are formed at every sweep);
// WPE: least waves per SIMD the register allocation must allow (0: any).
template <int L, int NW, bool JF, int UMAX, bool SPLIT, int WPE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NW * 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_pt(PtJob job, uint32_t k0, uint32_t k1)
{
    constexpr bool PREP = UMAX > 0;
    using G = Geo<L>;
    using Col = Column<L, JF, kColMajor, kColMajorOdd>;
    constexpr int NT = NW * 64;
    constexpr int JDW = G::jdw_odd(JF ? 2 : 1);
    extern __shared__ uint32_t lds[];
    const int T = job.T;
    const int tid = static_cast<int>(threadIdx.x);

    // run and group of this work group.  SPLIT: blocks are dealt round
    // robin to the eight XCDs, so blocks b and b + 8 share an XCD (and its
    // L2); the G groups of a run take blocks 8 apart.
    int run, g, TG;
    if constexpr (SPLIT) {
        const int b = static_cast<int>(blockIdx.x);
        const int j = b >> 3;
        TG = T / job.G;
        g = j % job.G;
        run = (j / job.G) * 8 + (b & 7);
        if (run >= job.n_runs) return;   // whole group, before any barrier
    } else {
        TG = T;
        g = 0;
        run = static_cast<int>(blockIdx.x);
    }
    const int w0 = g * TG;   // first walker of the group

    uint32_t *s_spin = lds;
    uint32_t *s_j = s_spin + TG * G::SPIN_DW;
    uint32_t *s_thr = s_j + JDW;
    int32_t *s_E = reinterpret_cast<int32_t *>(s_thr + T * kPtThr);
    int32_t *s_pos = s_E + T;
    int32_t *s_who = s_pos + T;
    int32_t *s_sw = s_who + T;
    uint32_t *s_thrx = reinterpret_cast<uint32_t *>(s_sw + T);
    const int mx = job.mx;

    const uint32_t chain = job.run0 + static_cast<uint32_t>(run);
    int8_t *spins = job.spins + static_cast<int64_t>(run) * T * G::N;

    // ---- set-up ---------------------------------------------------------
    for (int w = tid; w < TG * G::SPIN_DW; w += NT) s_spin[w] = 0u;
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
        if (p < 0 || p >= T) p = -1;   // out of range: not a permutation
        s_pos[tid] = p;
        s_who[tid] = -1;
    }
    load_couplings<L, JF, kColMajorOdd>(s_j, job.J, job.jenc, tid, NT);
    __syncthreads();
    if (tid < T && s_pos[tid] >= 0) s_who[s_pos[tid]] = tid;
    // a pos that is not a permutation of the slots leaves a slot without a
    // walker: every group of the run then takes the identity instead (so
    // every LDS index stays in range) and the status word records it
    if (__syncthreads_or(tid < T && s_who[tid] < 0)) {
        if (tid < T) {
            s_pos[tid] = tid;
            s_who[tid] = tid;
        }
        if (tid == 0 && job.status) atomicOr(job.status, 2);
    }
    {
        uint8_t *sb = reinterpret_cast<uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < TG * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            load_spins_one<L>(sb + wk * G::SPIN_DW * 4, q, job.init_random != 0,
                              spins + static_cast<int64_t>(w0 + wk) * G::N, static_cast<uint32_t>(w0 + wk), chain,
                              k0, k1);
        }
    }
    __syncthreads();
    for (int u = tid; u < TG * G::NC; u += NT) {
        const int wk = u / G::NC;
        const int col = u - wk * G::NC;
        atomicAdd(&s_E[w0 + wk], Col::column_energy_of(s_spin + wk * G::SPIN_DW, s_j, col));
    }
    __syncthreads();

    // prepared units: a lane keeps the same (walker, column) units for the
    // whole run (the launcher guarantees they number at most UMAX)
    constexpr int US = PREP ? UMAX : 1;
    typename Col::Unit un[US];
    int wks[US];
    bool act[US];
    if constexpr (PREP) {
#pragma unroll
        for (int i = 0; i < UMAX; ++i) {
            const int u = tid + i * NT;
            act[i] = u < TG * G::NC;
            const int ua = act[i] ? u : 0;
            const int wk = ua / G::NC;
            wks[i] = wk;
            un[i] = Col::make_unit(ua - wk * G::NC, static_cast<uint32_t>(w0 + wk), chain, k0, k1);
        }
    }
    bool dead = false;   // SPLIT: a wait gave up (wave 0 only)
    constexpr int NPRE = PREP ? pt_npre<L, NW, UMAX>() : 0;
    Rand4 drawn[NPRE > 0 ? NPRE : 1][G::C];   // colour-0 words of the coming step
    auto draw_colour0 = [&](uint32_t s) {
        if constexpr (NPRE > 0) {
#pragma unroll
            for (int i = 0; i < NPRE; ++i) {
                // one group per run: lanes without the unit skip it (20.36 ->
                // 19.91 ms on the PT workload); the split form draws on every
                // lane, which measured faster there (12.05 against 12.30 ms)
                if (!SPLIT && !act[i]) continue;
                const uint64_t q0 = philox_q0(un[i].hp, 2u * s);
#pragma unroll
                for (int m = 0; m < G::C; ++m) drawn[i][m] = philox_finish(un[i].pre[m], q0, k0, k1);
            }
        }
    };
    if (NPRE > 0 && job.n_steps > 0) draw_colour0(static_cast<uint32_t>(job.step0));

    // ---- steps ------------------------------------------------------------
    for (int ti = 0; ti < job.n_steps; ++ti) {
        const uint32_t t = static_cast<uint32_t>(job.step0 + ti);
        if constexpr (PREP) {
            // a unit's energy change over both colours goes to its walker in
            // one LDS atomic per step (the 64 lanes of a wave mostly share
            // one walker, so each such atomic is serialised)
            int32_t acc[UMAX];
            const uint32_t *tbl[UMAX];
#pragma unroll
            for (int i = 0; i < UMAX; ++i) {
                acc[i] = 0;
                tbl[i] = s_thr + s_pos[w0 + wks[i]] * kPtThr;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int i = 0; i < UMAX; ++i) {
                    if (!act[i]) continue;
                    uint32_t *rep = s_spin + wks[i] * G::SPIN_DW;
                    if (c == 0 && i < NPRE)
                        acc[i] += pt_colour0_drawn<L, Col>(rep, s_j, tbl[i], un[i], drawn[i < NPRE ? i : 0]);
                    else
                        acc[i] += Col::template metropolis_unit<true>(rep, s_j, tbl[i], c, un[i],
                                                                      2u * t + static_cast<uint32_t>(c), k0, k1);
                }
                if (c == 0) __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < UMAX; ++i)
                if (act[i] && acc[i] != 0) atomicAdd(&s_E[w0 + wks[i]], acc[i]);
            __syncthreads();
        } else {
            for (int c = 0; c < 2; ++c) {
                for (int u = tid; u < TG * G::NC; u += NT) {
                    const int wl = u / G::NC;
                    const int col = u - wl * G::NC;
                    const int wk = w0 + wl;
                    const int32_t dE = Col::template metropolis<true>(
                        s_spin + wl * G::SPIN_DW, s_j, s_thr + s_pos[wk] * kPtThr, c, col,
                        2u * t + static_cast<uint32_t>(c), static_cast<uint32_t>(wk), chain, k0, k1);
                    if (dE != 0) atomicAdd(&s_E[wk], dE);
                }
                __syncthreads();
            }
        }
        // Wave 0 (T <= 64 walkers, lane w holds walker w) runs the exchange
        // of ladder pairs (k, k+1), k = t mod 2, t mod 2 + 2, ..., lane k
        // deciding pair k.  Its random word follows from the counter alone,
        // so it is drawn before the energies are complete; the energies go
        // from lane to lane in registers.  Meanwhile the other waves draw
        // their colour-0 words of the next step.
        const int w = tid;
        const bool pair = w + 1 < T && ((w ^ static_cast<int>(t)) & 1) == 0;
        int32_t e = 0;
        uint32_t ux = 0;
        int a = 0, b = 0;
        if (tid < 64) {
            if (pair) {
                ux = philox10(static_cast<uint32_t>(w), t, 0xFFFFFFFFu, chain, k0, k1).w[0];
                a = s_who[w];
                b = s_who[w + 1];
            }
            if (w < T) e = s_E[w];
        }
        if constexpr (SPLIT) {
            // publish this group's energies, draw, then collect the other
            // groups' (every wave draws between the publishing and the wait)
            uint64_t *box = job.mbox + (static_cast<int64_t>(run) * 2 + (ti & 1)) * T;
            const uint32_t tag = static_cast<uint32_t>(ti) + 1u;
            const bool mine = w >= w0 && w < w0 + TG;
            if (tid < 64 && mine)
                __hip_atomic_store(box + w, (static_cast<uint64_t>(tag) << 32) | static_cast<uint32_t>(e),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (NPRE > 0 && ti + 1 < job.n_steps) draw_colour0(t + 1u);
            if (tid < 64) {
                bool gave_up = false;
                if (w < T && !mine && !dead) {
                    uint64_t v = 0;
                    for (int n = 0;; ++n) {
                        v = __hip_atomic_load(box + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (static_cast<uint32_t>(v >> 32) == tag) break;
                        if (n + 1 == kPtPollLimit) {
                            gave_up = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    e = static_cast<int32_t>(static_cast<uint32_t>(v));
                    s_E[w] = e;
                }
                if (__any(gave_up)) {
                    if (!dead && w == 0) atomicOr(job.status, 1);
                    dead = true;
                }
            }
        } else {
            if (NPRE > 0 && tid >= 64 && ti + 1 < job.n_steps) draw_colour0(t + 1u);
        }
        if (tid < 64) {
            const int32_t ea = __shfl(e, a, 64), eb = __shfl(e, b, 64);
            if (pair) {
                const int32_t D = ea - eb;
                bool acc = D <= 0;
                if (!acc) {
                    const int32_t m = D / 2;
                    if (m <= mx)
                        acc = ux < s_thrx[w * mx + (m - 1)];
                    else
                        acc = (m <= job.M) && (ux < job.thrx[static_cast<int64_t>(w) * job.M + (m - 1)]);
                }
                if (acc) {
                    s_who[w] = b;
                    s_who[w + 1] = a;
                    s_pos[b] = w;
                    s_pos[a] = w + 1;
                    s_sw[w] += 1;
                }
            }
            // minimum energy of the step (group 0 of a split run)
            if (job.emin_trace && g == 0) {
                int32_t mn = w < T ? e : 0x7FFFFFFF;
                for (int off = 32; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
                if (w == 0) job.emin_trace[static_cast<int64_t>(run) * job.n_steps + ti] = mn;
            }
        }
        if constexpr (!SPLIT)
            if (NPRE > 0 && tid < 64 && ti + 1 < job.n_steps) draw_colour0(t + 1u);
        __syncthreads();
    }

    // ---- write-back ---------------------------------------------------------
    {
        const uint8_t *sb = reinterpret_cast<const uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < TG * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            store_spins_one<L>(sb + wk * G::SPIN_DW * 4, q, spins + static_cast<int64_t>(w0 + wk) * G::N);
        }
    }
    // group 0 holds every walker's final energy (the last step's mailbox)
    if (g == 0 && tid < T) {
        job.energy[run * T + tid] = s_E[tid];
        job.pos[run * T + tid] = s_pos[tid];
        if (job.swap_acc && tid + 1 < T) job.swap_acc[run * (T - 1) + tid] += static_cast<uint32_t>(s_sw[tid]);
    }
}

// Zeroes a split launch's mailbox (n words; tags start at 1) and the status
// word (a template, so that both entry points' translation units may hold it)
template <int Unused = 0>
__global__ __launch_bounds__(256) void k_pt_split_clear(uint64_t *mbox, int64_t n, int32_t *status)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) mbox[i] = 0;
    if (i == 0) status[0] = 0;
}

// Launch T-walker runs with G work groups each (G = 1 without SPLIT) and NW
// waves per group; `lds_cap` bounds one group's LDS (a fraction of the
// CU's 160 KB lets several groups share a CU).  SPLIT launches
// ceil(n_runs/8) * 8 * G groups.
template <int L, int NW, int UMAX, bool SPLIT, int WPE>
static int launch_pt_cfg(PtJob job, int n_runs, uint32_t k0, uint32_t k1, hipStream_t stream, const char *who,
                         size_t lds_cap = 160 * 1024)
{
    using Cfg = PtCfg<L>;
    auto kern = k_pt<L, NW, Cfg::JF, UMAX, SPLIT, WPE>;
    lds_cap = std::min(lds_cap, lds_dynamic_cap(reinterpret_cast<const void *>(kern)));
    const int TG = job.T / job.G;
    const size_t base = pt_lds_bytes<L, Cfg::JF>(TG, job.T, 0);
    if (base > lds_cap)
        return fail(SG_EUNSUPPORTED, "%s: L = %d with %d walkers per group needs %zu bytes of LDS", who, L, TG, base);
    // the exchange-table prefix held in LDS: up to 128 entries per pair,
    // as many as the LDS left over allows (later entries are read from HBM)
    job.mx = static_cast<int32_t>(std::min<size_t>({static_cast<size_t>(job.M), 128,
                                                   (lds_cap - base) / (4 * static_cast<size_t>(job.T - 1))}));
    const size_t bytes = pt_lds_bytes<L, Cfg::JF>(TG, job.T, job.mx);
    const int units = TG * Geo<L>::NC;
    if (UMAX > 0 && (units + NW * 64 - 1) / (NW * 64) > UMAX)
        return fail(SG_EUNSUPPORTED, "%s: %d units per colour exceed %d lanes x %d prepared units", who, units,
                    NW * 64, UMAX);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (err != hipSuccess) return fail(SG_EDEVICE, "%s: LDS attribute: %s", who, hipGetErrorString(err));
    const int blocks = SPLIT ? ((n_runs + 7) / 8) * 8 * job.G : n_runs;
    if constexpr (SPLIT) {
        // every group of the launch must be resident at once: a group waits
        // on the other groups of its run
        int dev = 0, n_cu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), NW * 64,
                                                         bytes) != hipSuccess)
            return fail(SG_EDEVICE, "%s: occupancy query failed", who);
        if (static_cast<int64_t>(blocks) > static_cast<int64_t>(per_cu) * n_cu)
            return fail(SG_EUNSUPPORTED, "%s: %d work groups exceed the %d x %d the device holds at once", who, blocks,
                        per_cu, n_cu);
    }
    (void)hipGetLastError();
    if (job.status) {
        // after every check: the mailbox (split form) and the status word
        const int64_t n = SPLIT ? static_cast<int64_t>(n_runs) * 2 * job.T : 0;
        hipLaunchKernelGGL(k_pt_split_clear<0>, dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + 255) / 256))),
                           dim3(256), 0, stream, job.mbox, n, job.status);
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NW * 64), bytes, stream, job, k0, k1);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "%s: launch failed: %s", who, hipGetErrorString(err));
    return SG_OK;
}

// one-group-per-run launch (and the split form's default): prepared units
// when they fit the register budget of NW waves
template <int L, int NW, bool SPLIT>
static int launch_pt_nw(const PtJob &job, int n_runs, uint32_t k0, uint32_t k1, hipStream_t stream, const char *who)
{
    constexpr int UM = pt_umax<L, NW>();
    const int units = job.T / job.G * Geo<L>::NC;
    const int upl = (units + NW * 64 - 1) / (NW * 64);
    if (UM > 0 && upl <= UM) return launch_pt_cfg<L, NW, UM, SPLIT, 0>(job, n_runs, k0, k1, stream, who);
    return launch_pt_cfg<L, NW, 0, SPLIT, 0>(job, n_runs, k0, k1, stream, who);
}

template <int L, bool SPLIT>
static int launch_pt(const PtJob &job, int n_runs, int nw, uint32_t k0, uint32_t k1, hipStream_t stream,
                     const char *who)
{
    switch (nw) {
    case 4: return launch_pt_nw<L, 4, SPLIT>(job, n_runs, k0, k1, stream, who);
    case 8: return launch_pt_nw<L, 8, SPLIT>(job, n_runs, k0, k1, stream, who);
    case 12: return launch_pt_nw<L, 12, SPLIT>(job, n_runs, k0, k1, stream, who);
    default: return launch_pt_nw<L, 16, SPLIT>(job, n_runs, k0, k1, stream, who);
    }
}

// Host validation shared by both entry points; fills job from the arguments.
inline int pt_prepare(const sg_instance *inst, const sg_pt_args *args, const uint32_t *thr, const uint32_t *thrx,
                      int8_t *spins, int32_t *energy_out, int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc,
                      const char *who, PtJob &job)
{
    if (!inst || !args) return fail(SG_EINVAL, "%s: NULL instance or args", who);
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "%s: L = %d must be even in [4, %d]", who, inst->L, SG_MAX_L);
    if (!inst->J && !inst->jenc) return fail(SG_EINVAL, "%s: instance has no couplings", who);
    if (!thr || !thrx || !spins || !energy_out || !pos) return fail(SG_EINVAL, "%s: NULL array", who);
    if (args->n_runs < 1 || args->n_steps < 1)
        return fail(SG_EINVAL, "%s: n_runs = %d, n_steps = %d", who, args->n_runs, args->n_steps);
    if (args->T < 2 || args->T > SG_PT_MAX_T) return fail(SG_EINVAL, "%s: T = %d outside [2, %d]", who, args->T, SG_PT_MAX_T);
    if (args->K < 1 || args->K > SG_K_MAX || args->M < 1) return fail(SG_EINVAL, "%s: K = %d, M = %d", who, args->K, args->M);
    if (args->step0 < 0 || static_cast<int64_t>(args->step0) + args->n_steps > (1 << 30))
        return fail(SG_ERANGE, "%s: steps must stay below 2^30", who);
    if (static_cast<uint64_t>(args->run0) + static_cast<uint64_t>(args->n_runs) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "%s: run counter words overflow", who);
    if ((reinterpret_cast<uintptr_t>(spins) & 3u) != 0) return fail(SG_EINVAL, "%s: spins must be 4-byte aligned", who);
    job = PtJob{};
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
    job.n_runs = args->n_runs;
    job.G = 1;
    return SG_OK;
}

template <bool SPLIT>
inline int pt_dispatch(int L, const PtJob &job, int n_runs, int nw, uint32_t k0, uint32_t k1, hipStream_t st,
                       const char *who)
{
    switch (L) {
    case 4: return launch_pt<4, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 6: return launch_pt<6, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 8: return launch_pt<8, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 10: return launch_pt<10, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 12: return launch_pt<12, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 14: return launch_pt<14, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    case 16: return launch_pt<16, SPLIT>(job, n_runs, nw, k0, k1, st, who);
    default: return fail(SG_EUNSUPPORTED, "%s: L = %d is above the LDS-resident PT range", who, L);
    }
}

}  // namespace sg
