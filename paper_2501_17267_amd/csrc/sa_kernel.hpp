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
    uint32_t k0, k1;        // Philox key (batched launches)
};

// Launch shape per lattice size: RPW replicas per group, NW waves, JF =
// keep both coupling encodings (E, F) in LDS.  Chosen so that
// RPW * L^2/2 column units spread evenly over NW*64 lanes and the group's
// LDS (couplings + RPW spin blocks) leaves room for a second group where
// possible.
template <int L>
struct SaCfg;
template <> struct SaCfg<4> { static constexpr int RPW = 16, NW = 2; static constexpr bool JF = true; };
template <> struct SaCfg<6> { static constexpr int RPW = 32, NW = 3; static constexpr bool JF = true; };
template <> struct SaCfg<8> { static constexpr int RPW = 16, NW = 4; static constexpr bool JF = true; };
template <> struct SaCfg<10> { static constexpr int RPW = 32, NW = 5; static constexpr bool JF = true; };
template <> struct SaCfg<12> { static constexpr int RPW = 16, NW = 6; static constexpr bool JF = true; };
template <> struct SaCfg<14> { static constexpr int RPW = 32, NW = 7; static constexpr bool JF = false; };
template <> struct SaCfg<16> { static constexpr int RPW = 16, NW = 8; static constexpr bool JF = true; };
template <> struct SaCfg<18> { static constexpr int RPW = 8, NW = 7; static constexpr bool JF = false; };
template <> struct SaCfg<20> { static constexpr int RPW = 8, NW = 5; static constexpr bool JF = false; };
template <> struct SaCfg<22> { static constexpr int RPW = 4, NW = 8; static constexpr bool JF = false; };
template <> struct SaCfg<24> { static constexpr int RPW = 4, NW = 9; static constexpr bool JF = false; };

template <int L, int RPW, int NW, bool JF, bool TRACK>
__device__ void sa_group(const SaJob &job, int group, uint32_t k0, uint32_t k1)
{
    using G = Geo<L>;
    using Col = Column<L, JF>;
    constexpr int NT = NW * 64;
    constexpr int JDW = JF ? G::JDW_EF : G::JDW_E;
    __shared__ uint32_t s_spin[RPW * G::SPIN_DW];
    __shared__ uint32_t s_j[JDW];
    __shared__ uint32_t s_thr[2][256];
    __shared__ int32_t s_dE[2][RPW];
    __shared__ int32_t s_E[RPW];

    const int tid = static_cast<int>(threadIdx.x);
    const int r_first = group * RPW;
    const int nact = min(RPW, job.n_rep - r_first);
    constexpr bool track = TRACK;

    // ---- set-up ---------------------------------------------------------
    for (int w = tid; w < RPW * G::SPIN_DW; w += NT) s_spin[w] = 0u;
    for (int w = tid; w < 2 * 256; w += NT) {
        const int e = w & 255;
        uint32_t v = 0u;
        if (e <= 48) v = 0xFFFFFFFFu;
        else if (e - 49 < job.K) v = job.thr[e - 49];
        s_thr[w >> 8][e] = v;
    }
    if (tid < RPW) {
        s_dE[0][tid] = 0;
        s_dE[1][tid] = 0;
        s_E[tid] = 0;
    }
    load_couplings<L, JF>(s_j, job.J, job.jenc, tid, NT);
    __syncthreads();
    {
        uint8_t *sb = reinterpret_cast<uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < nact * Q; w += NT) {
            const int rl = w / Q;
            const int q = w - rl * Q;
            const int r = r_first + rl;
            load_spins_one<L>(sb + rl * G::SPIN_DW * 4, q, job.init_random != 0,
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
            uint32_t own[G::C], kb[G::C];
            Col::fields(s_spin + rl * G::SPIN_DW, s_j, 0, col, own, kb);
            atomicAdd(&s_E[rl], Col::column_energy(kb));
        }
        __syncthreads();
    }
    int32_t best = 0x7FFFFFFF;

    // ---- sweeps ---------------------------------------------------------
    for (int si = 0; si < job.n_sweeps; ++si) {
        const int buf = si & 1;
        const uint32_t s_abs = static_cast<uint32_t>(job.sweep0 + si);
        if (si + 1 < job.n_sweeps && tid < job.K)
            s_thr[buf ^ 1][49 + tid] = job.thr[static_cast<int64_t>(si + 1) * job.K + tid];
        for (int c = 0; c < 2; ++c) {
            for (int u = tid; u < nact * G::NC; u += NT) {
                const int rl = u / G::NC;
                const int col = u - rl * G::NC;
                const uint32_t rep_word = job.rep0 + static_cast<uint32_t>(r_first + rl);
                const int32_t dE = Col::template metropolis<TRACK>(s_spin + rl * G::SPIN_DW, s_j, s_thr[buf], c, col,
                                                   2u * s_abs + static_cast<uint32_t>(c), rep_word,
                                                   job.chain, k0, k1);
                if (TRACK && dE != 0) atomicAdd(&s_dE[buf][rl], dE);
            }
            __syncthreads();
        }
        if (track && tid < nact) {
            s_E[tid] += s_dE[buf][tid];
            s_dE[buf][tid] = 0;
            best = min(best, s_E[tid]);
        }
    }

    // ---- final energy and write-back -----------------------------------
    if (tid < RPW) s_dE[0][tid] = 0;
    __syncthreads();
    for (int u = tid; u < nact * G::NC; u += NT) {
        const int rl = u / G::NC;
        const int col = u - rl * G::NC;
        uint32_t own[G::C], kb[G::C];
        Col::fields(s_spin + rl * G::SPIN_DW, s_j, 0, col, own, kb);
        atomicAdd(&s_dE[0][rl], Col::column_energy(kb));
    }
    {
        const uint8_t *sb = reinterpret_cast<const uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < nact * Q; w += NT) {
            const int rl = w / Q;
            const int q = w - rl * Q;
            store_spins_one<L>(sb + rl * G::SPIN_DW * 4, q,
                               job.spins + static_cast<int64_t>(r_first + rl) * G::N);
        }
    }
    __syncthreads();
    if (tid < nact) {
        job.energy[r_first + tid] = s_dE[0][tid];
        if (track && job.emin) job.emin[r_first + tid] = best;
    }
}

}  // namespace sg
