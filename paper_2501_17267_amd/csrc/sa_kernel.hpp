// sa_kernel.hpp -- body of one simulated-annealing work group (shared by the
// per-instance and the batched launches).
#pragma once

#include "sweep.hpp"

namespace sg {

// One annealing job: an instance, a replica range and a schedule slice.
struct SaJob {
    const int8_t *J;        // natural-order couplings [6][N] (or NULL with jenc)
    const uint32_t *jenc;   // encoded couplings or NULL
    const uint32_t *thr;    // [n_sweeps][K]
    int8_t *spins;          // [n_rep][N]
    int32_t *energy;        // [n_rep]
    int32_t *emin;          // [n_rep] or NULL
    uint32_t chain;
    uint32_t rep0;
    int32_t n_rep;
    int32_t n_sweeps;
    int32_t sweep0;
    int32_t K;
    int32_t init_random;
    int32_t pad;
    uint32_t k0, k1;        // Philox key
    uint32_t *workspace;    // global spin blocks when the lattice is not LDS-resident
};

// Where the couplings live during the anneal.
enum : int {
    kJLdsEF = 0,    // LDS, both encodings E = J + 8 and F = 8 - J
    kJLdsE = 1,     // LDS, E only (F = 16 - E computed per use)
    kJGlobalEF = 2, // streamed from the encoded HBM buffer (jenc), E and F
    kJLds3E = 3     // LDS, E of the three forward directions (backward ones from the neighbours)
};

// A replica group inside a job (batched launches: one work group each).
struct Group {
    int32_t job;    // index into the job table
    int32_t group;  // replica group inside the job
};

template <int L, int RPW, int NW, int JM, bool SPIN_LDS, bool TRACK>
__device__ void sa_group(const SaJob &job, int group, uint32_t k0, uint32_t k1)
{
    using G = Geo<L>;
    constexpr bool JF = (JM != kJLdsE && JM != kJLds3E);
    // LDS arrays column-major (spin columns of 3, 5 or 6 dwords split in
    // two planes), HBM arrays dword-major (coalesced)
    constexpr int SLAY = SPIN_LDS ? (G::SPLIT_COLUMNS ? kColSplit : kColMajor) : kDwordMajor;
    constexpr int JLAY = (JM == kJGlobalEF) ? kDwordMajor : (JM == kJLds3E ? kFwd3 : kColMajor);
    using Col = Column<L, JF, SLAY, JLAY>;
    constexpr int NT = NW * 64;
    constexpr int JDW = (JM == kJGlobalEF) ? 0 : (JM == kJLds3E ? G::JDW_3E : (JF ? G::JDW_EF : G::JDW_E));
    constexpr int SDW = SPIN_LDS ? RPW * G::SPIN_DW : 0;
    // One LDS block: the two threshold tables first (fixed addresses 0 and
    // 256 bytes, so table lookups need no base register), then per-replica
    // energy slots, the encoded couplings and the replicas' spins (the last
    // two only when they are LDS-resident).
    constexpr int OFF_THR = 0;
    constexpr int OFF_DE = 2 * kThrEntries;
    constexpr int OFF_E = OFF_DE + 2 * RPW;
    // couplings and spins start on a 16-byte boundary so that column reads
    // are single 128-bit LDS accesses whatever RPW is
    constexpr int OFF_J = (OFF_E + RPW + 3) & ~3;
    constexpr int OFF_SPIN = OFF_J + JDW;
    constexpr int TOTAL = OFF_SPIN + SDW;
    __shared__ uint32_t lds[TOTAL];
    uint32_t *s_thr0 = lds + OFF_THR;
    uint32_t *s_thr1 = lds + OFF_THR + kThrEntries;
    int32_t *s_dE0 = reinterpret_cast<int32_t *>(lds + OFF_DE);
    int32_t *s_dE1 = s_dE0 + RPW;
    int32_t *s_E = reinterpret_cast<int32_t *>(lds + OFF_E);
    const int tid = static_cast<int>(threadIdx.x);
    const int r_first = group * RPW;
    const uint32_t *s_j = (JM == kJGlobalEF) ? job.jenc : lds + OFF_J;
    uint32_t *s_spin = SPIN_LDS ? lds + OFF_SPIN
                                : job.workspace + static_cast<int64_t>(r_first) * G::SPIN_DW;
    const int nact = min(RPW, job.n_rep - r_first);
    constexpr bool track = TRACK;

    // ---- set-up ---------------------------------------------------------
    for (int w = tid; w < RPW * G::SPIN_DW; w += NT) s_spin[w] = 0u;
    for (int w = tid; w < 2 * kThrEntries; w += NT) {
        const int e = w % kThrEntries;
        s_thr0[w] = thr_entry(job.thr, job.K, e);
    }
    if (tid < RPW) {
        s_dE0[tid] = 0;
        s_dE1[tid] = 0;
        s_E[tid] = 0;
    }
    if (JM != kJGlobalEF) load_couplings<L, JF, JLAY>(lds + OFF_J, job.J, job.jenc, tid, NT);
    __syncthreads();
    {
        uint8_t *sb = reinterpret_cast<uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < nact * Q; w += NT) {
            const int rl = w / Q;
            const int q = w - rl * Q;
            const int r = r_first + rl;
            load_spins_one<L, SLAY>(sb + rl * G::SPIN_DW * 4, q, job.init_random != 0,
                              job.spins + static_cast<int64_t>(r) * G::N,
                              job.rep0 + static_cast<uint32_t>(r), job.chain, k0, k1);
        }
    }
    __syncthreads();

    // initial energy (only needed for the best-seen energy)
    if (track) {
        for (int u = tid; u < nact * G::NC; u += NT) {
            const int rl = u / G::NC;
            const int col = u - rl * G::NC;
            atomicAdd(&s_E[rl], Col::column_energy_of(s_spin + rl * G::SPIN_DW, s_j, col));
        }
        __syncthreads();
    }
    int32_t best = 0x7FFFFFFF;

    // ---- sweeps ---------------------------------------------------------
    // Two threshold tables at fixed LDS addresses: even sweeps read s_thr0,
    // odd sweeps s_thr1 (the loop is unrolled by two so that each table's
    // address is a compile-time constant); the row of sweep si+1 is written
    // into the other table while sweep si runs.
    // Columns held whole in registers: each lane's units (column, replica)
    // are fixed for the anneal, so their neighbour columns and the
    // sweep-independent part of their Philox calls are prepared once.
    // Only where that state (4 words per dword + 8 per unit) fits in the
    // registers the sweep leaves free: 40 per lane, or 60 at 9 to 12 waves
    // (three waves per SIMD: such a group has the compute unit's registers
    // to itself, 168 per lane); shapes with more units per lane keep the
    // per-sweep path.
    constexpr int UPL = (RPW * G::NC + NT - 1) / NT;
    constexpr int kPrepRegs = (NW >= 9 && NW <= 12) ? 60 : 40;
    constexpr bool kPrep = !Col::kStream && UPL * (4 * G::C + 8) <= kPrepRegs;
    typename Col::Unit un[kPrep ? UPL : 1];
    int rls[kPrep ? UPL : 1];
    bool act[kPrep ? UPL : 1];
    if constexpr (kPrep) {
#pragma unroll
        for (int i = 0; i < UPL; ++i) {
            const int u = tid + i * NT;
            act[i] = u < nact * G::NC;
            const int ua = act[i] ? u : 0;
            const int rl = ua / G::NC;
            const int col = ua - rl * G::NC;
            rls[i] = rl;
            un[i] = Col::make_unit(col, job.rep0 + static_cast<uint32_t>(r_first + rl), job.chain, k0, k1);
        }
    }

    auto sweep = [&](int si, const uint32_t *thr_now, uint32_t *thr_next) {
        const uint32_t s_abs = static_cast<uint32_t>(job.sweep0 + si);
        if (si + 1 < job.n_sweeps && tid < job.K)
            thr_next[kKbBias + 1 + tid] = job.thr[static_cast<int64_t>(si + 1) * job.K + tid];
        if constexpr (kPrep) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int i = 0; i < UPL; ++i) {
                    if (!act[i]) continue;
                    const int32_t dE = Col::template metropolis_unit<TRACK>(
                        s_spin + rls[i] * G::SPIN_DW, s_j, thr_now, c, un[i], 2u * s_abs + static_cast<uint32_t>(c), k0,
                        k1);
                    if (TRACK && dE != 0) atomicAdd(&((si & 1) ? s_dE1 : s_dE0)[rls[i]], dE);
                }
                __syncthreads();
            }
        } else {
            for (int c = 0; c < 2; ++c) {
                for (int u = tid; u < nact * G::NC; u += NT) {
                    const int rl = u / G::NC;
                    const int col = u - rl * G::NC;
                    const uint32_t rep_word = job.rep0 + static_cast<uint32_t>(r_first + rl);
                    const int32_t dE = Col::template metropolis<TRACK>(
                        s_spin + rl * G::SPIN_DW, s_j, thr_now, c, col, 2u * s_abs + static_cast<uint32_t>(c),
                        rep_word, job.chain, k0, k1);
                    if (TRACK && dE != 0) atomicAdd(&((si & 1) ? s_dE1 : s_dE0)[rl], dE);
                }
                __syncthreads();
            }
        }
        if (track && tid < nact) {
            int32_t *acc = (si & 1) ? s_dE1 : s_dE0;
            s_E[tid] += acc[tid];
            acc[tid] = 0;
            best = min(best, s_E[tid]);
        }
    };
    for (int si = 0; si < job.n_sweeps; si += 2) {
        sweep(si, s_thr0, s_thr1);
        if (si + 1 < job.n_sweeps) sweep(si + 1, s_thr1, s_thr0);
    }

    // ---- final energy and write-back -----------------------------------
    if (tid < RPW) s_dE0[tid] = 0;
    __syncthreads();
    for (int u = tid; u < nact * G::NC; u += NT) {
        const int rl = u / G::NC;
        const int col = u - rl * G::NC;
        atomicAdd(&s_dE0[rl], Col::column_energy_of(s_spin + rl * G::SPIN_DW, s_j, col));
    }
    {
        const uint8_t *sb = reinterpret_cast<const uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < nact * Q; w += NT) {
            const int rl = w / Q;
            const int q = w - rl * Q;
            store_spins_one<L, SLAY>(sb + rl * G::SPIN_DW * 4, q,
                               job.spins + static_cast<int64_t>(r_first + rl) * G::N);
        }
    }
    __syncthreads();
    if (tid < nact) {
        job.energy[r_first + tid] = s_dE0[tid];
        if (track && job.emin) job.emin[r_first + tid] = best;
    }
}

}  // namespace sg
