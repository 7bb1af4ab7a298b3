// pticm.hip -- parallel tempering with isoenergetic cluster moves (App. D,
// PT+ICM; the cluster move is Houdayer's two-replica move as combined with
// PT by Zhu, Ochoa and Katzgraber) and its C-ABI entry point.
//
// One work group runs one run: two copies of a T-slot ladder (2T walkers),
// all LDS-resident in the colour column layout.  A step is the sweep of
// every walker, then for every slot k >= icm_from one cluster move between
// the two walkers at slot k, then the even/odd exchanges inside each copy.
// The moves of different slots touch different walkers, so each slot's move
// is run by one wave on its own, with no block barrier: the disagreement
// of the two walkers and the cluster are held as bits (one dword per double
// column, see IcmBits), a wave prefix count over (colour, column, height)
// picks the seed, the cluster grows breadth first (every site of the
// frontier at once, one hop per round) until a round adds nothing, and
// both walkers then flip it.
#include <algorithm>

#include "common.hpp"
#include "sweep.hpp"
#include "variants.hpp"

namespace sg {

struct PtIcmJob {
    const int8_t *J;
    const uint32_t *jenc;
    const uint32_t *thr;    // [T][K]
    const uint32_t *thrx;   // [T-1][M]
    int8_t *spins;          // [n_runs][2T][N]
    int32_t *energy;        // [n_runs][2T]
    int32_t *pos;           // [n_runs][2T]
    int32_t *emin_trace;    // [n_runs][n_steps] or NULL
    uint32_t *swap_acc;     // [n_runs][2(T-1)] or NULL
    int32_t *icm_flipped;   // [n_runs][n_steps] or NULL
    uint32_t run0;
    int32_t T, n_steps, step0, K, M, icm_from, init_random;
    int32_t mx;             // exchange-table entries per ladder pair held in LDS
};

constexpr int kIcmNW = 12;          // 768 lanes per run
constexpr int kIcmThr = kThrEntries;
constexpr int kIcmMx = 128;        // exchange-table entries per pair staged in LDS (at most)

// One slot's sites as bits.  Item col is the double column of index col:
// both colour columns, i.e. the sites with x in {2k, 2k+1} at one y, every
// z.  Its dword holds the colour-0 sites at bits z = 0..L-1 and the
// colour-1 sites at bits L + z.  Every bond joins the two colours, so the
// neighbours of a site are bits of the other half: z +- 1 and the x link
// inside the item in the same dword; the other x link (to item k-1 for even
// x, k+1 for odd x) and the y links in the neighbouring items' dwords.
template <int L>
struct IcmBits {
    static_assert(L <= 16, "a double column must fit a dword");
    static constexpr int NC = Geo<L>::NC;
    static constexpr int NI = (NC + 63) / 64;   // items per lane
    static constexpr int ROW = 64 * NI;         // a wave's cluster row: one dword per lane and item
    static constexpr uint32_t FULL = L == 16 ? 0xFFFFFFFFu : (1u << (2 * L)) - 1u;
    static constexpr uint32_t LOW = 1u | (1u << L);                       // z = 0 of each half
    static constexpr uint32_t HIGH = (1u << (L - 1)) | (1u << (2 * L - 1));  // z = L-1 of each half
    // the two halves exchanged
    __device__ static uint32_t swap(uint32_t v) { return ((v >> L) | (v << L)) & FULL; }
    // bit z of each half to z + 1, periodic in L
    __device__ static uint32_t up(uint32_t v) { return ((v << 1) & ~LOW & FULL) | ((v >> (L - 1)) & LOW); }
    // bit z of each half to z - 1, periodic in L
    __device__ static uint32_t down(uint32_t v) { return ((v >> 1) & ~HIGH) | ((v << (L - 1)) & HIGH); }
    // the four 0x00/0xFF bytes of a column dword as four bits
    __device__ static uint32_t gather4(uint32_t v) { return ((v & 0x01010101u) * 0x01020408u) >> 24; }
    // four bits as 0x00/0xFF bytes
    __device__ static uint32_t spread4(uint32_t b)
    {
        const uint32_t t = (b * 0x00204081u) & 0x01010101u;   // b < 16: a 24-bit product
        return (t << 8) - t;
    }
    // bits of column dword m inside a half (the tail dword has fewer heights)
    static constexpr uint32_t dword_bits(int m) { return L - 4 * m >= 4 ? 0xFu : (1u << (L - 4 * m)) - 1u; }
};

// LDS of one run: walkers, couplings, thresholds, ladder words, the
// nonzero-coupling masks (bytes, then bits) and one cluster row per wave
template <int L, bool JF>
constexpr size_t pticm_lds_bytes(int T, int mx)
{
    using G = Geo<L>;
    const size_t W = 2 * static_cast<size_t>(T);
    return (W * G::SPIN_DW + G::jdw_odd(JF ? 2 : 1) + static_cast<size_t>(T) * kIcmThr + 3 * W +
            2 * (static_cast<size_t>(T) - 1) + static_cast<size_t>(T) + 6 * static_cast<size_t>(G::SPIN_DW) +
            7 * static_cast<size_t>(G::NC) + static_cast<size_t>(kIcmNW) * IcmBits<L>::ROW +
            static_cast<size_t>(T - 1) * static_cast<size_t>(mx)) * 4;
}

// Directions of the link masks (receiving site's coupling nonzero), kept
// with the halves exchanged so that they apply to the sending side's bits:
// +z, -z, the x link inside the item, -x to item k-1, +x to item k+1, +y, -y
enum : int { kLmZp = 0, kLmZm, kLmXin, kLmXm, kLmXp, kLmYp, kLmYm, kLmN };

// hops inside an item per breadth-first round, after the hop that reads the
// neighbouring items
constexpr int kIcmInnerHops = 1;

// wave-wide prefix sums and sums (the device library's, on DPP lane moves
// instead of LDS round trips); every lane of the wave must take part
extern "C" __device__ int __ockl_wfscan_add_i32(int, bool);
extern "C" __device__ int __ockl_wfred_add_i32(int);
extern "C" __device__ int __ockl_wfred_min_i32(int);

// exclusive prefix sum over the lanes of a wave, and the wave total
__device__ __forceinline__ int wave_excl_scan(int v, int &total)
{
    const int incl = __ockl_wfscan_add_i32(v, true);
    total = __builtin_amdgcn_readlane(incl, 63);
    return incl - v;
}

__device__ __forceinline__ int wave_sum(int v) { return __ockl_wfred_add_i32(v); }

// position of the j-th set bit (j counted from 0) of f
__device__ __forceinline__ uint32_t nth_bit(uint32_t f, int j)
{
    // halving search: the j-th set bit lies in the low half of the window
    // when the low half holds more than j set bits, else in the high half
    // (j < popcount(f) at every call)
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const int c = __popc(f & ((1u << w) - 1u));
        if (j >= c) {
            j -= c;
            f >>= w;
            pos += w;
        }
    }
    return 1u << pos;
}

// The cluster move of one slot between walkers wa and wb (two copies at the
// same ladder slot k), run by one whole wave.  lm: link masks [kLmN][NC];
// wcl: the wave's cluster row [IcmBits::ROW].  The lanes read each other's
// items through wcl, so the growth loop keeps the whole wave together: no
// lane branches inside it, every lane stores all its slots every round.  Writes the two walkers' new energies
// and the cluster size (0 when the walkers agree everywhere).
template <int L, bool JF>
__device__ void icm_move_wave(uint32_t *s_spin, const uint32_t *s_j, const uint32_t *lm, uint32_t *wcl, int wa,
                              int wb, int k, uint32_t t, uint32_t chain, uint32_t k0, uint32_t k1, int lane,
                              int32_t *s_E, int32_t *size_out)
{
    using G = Geo<L>;
    using B = IcmBits<L>;
    using Col = Column<L, JF, kColMajor, kColMajorOdd>;
    constexpr int NC = G::NC, C = G::C, SDW = G::SPIN_DW, NI = B::NI;
    uint32_t *sa = s_spin + wa * SDW;
    uint32_t *sb = s_spin + wb * SDW;
    // the seed's random word follows from the counter alone: drawn first,
    // its arithmetic beside the loads below
    const Rand4 uu = philox10(static_cast<uint32_t>(k), t, 0xFFFFFFFEu, chain, k0, k1);
    // 1. the disagreeing sites as bits
    uint32_t q[NI], cl[NI];
    int n0[NI], n1[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int I = lane + 64 * i;
        q[i] = 0u;
        if (I < NC) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int m = 0; m < C; ++m) {
                    const int w = (c * NC + I) * C + m;
                    q[i] |= (B::gather4(sa[w] ^ sb[w]) & B::dword_bits(m)) << (c * L + 4 * m);
                }
        }
        n0[i] = __popc(q[i] & ((1u << L) - 1u));
        n1[i] = __popc(q[i] >> L);
    }
    // 2. the seed: the r-th disagreeing site in the order (colour, column,
    // height), r drawn from the slot's counter
    int p0[NI], p1[NI], tot = 0, N0 = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        p0[i] = N0 + wave_excl_scan(n0[i], tot);
        N0 += tot;
    }
    int N1 = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        p1[i] = N0 + N1 + wave_excl_scan(n1[i], tot);
        N1 += tot;
    }
    const int n = N0 + N1;
    if (n == 0) {
        if (lane == 0) *size_out = 0;
        return;
    }
    const int r = static_cast<int>((static_cast<uint64_t>(uu.w[0]) * static_cast<uint64_t>(n)) >> 32);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        cl[i] = 0u;
        if (r >= p0[i] && r < p0[i] + n0[i]) cl[i] = nth_bit(q[i] & ((1u << L) - 1u), r - p0[i]);
        if (r >= p1[i] && r < p1[i] + n1[i]) cl[i] = nth_bit(q[i] >> L, r - p1[i]) << L;
    }
    // 3. growth: a round gives every disagreeing site linked to the cluster
    // to it; the rounds end at the connected component of the seed
    uint32_t msk[NI][kLmN];
    int nxm[NI], nxp[NI], nyp[NI], nym[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int I = lane + 64 * i;
        const int Ia = I < NC ? I : 0;
#pragma unroll
        for (int d = 0; d < kLmN; ++d) msk[i][d] = I < NC ? lm[d * NC + Ia] : 0u;
        const typename Col::Nbr nb = Col::neighbours(0, Ia);
        nxm[i] = nb.xm;
        nxp[i] = nb.xp;
        nyp[i] = nb.yp;
        nym[i] = nb.ym;
        wcl[I] = cl[i];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (;;) {
        uint32_t grown = 0;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const uint32_t a = wcl[nxm[i]], b = wcl[nxp[i]], c = wcl[nyp[i]], d = wcl[nym[i]];
            const uint32_t own = cl[i];
            uint32_t A = (B::down(own) & msk[i][kLmZp]) | (B::up(own) & msk[i][kLmZm]) | (own & msk[i][kLmXin]);
            A |= (a & msk[i][kLmXm]) | (b & msk[i][kLmXp]) | (c & msk[i][kLmYp]) | (d & msk[i][kLmYm]);
            const uint32_t nw = B::swap(A) & q[i] & ~own;
            // then kIcmInnerHops more hops inside the item (z links and the
            // inner x link), which need no other lane
            uint32_t cur = own | nw;
#pragma unroll
            for (int h = 0; h < kIcmInnerHops; ++h)
                cur |= B::swap((B::down(cur) & msk[i][kLmZp]) | (B::up(cur) & msk[i][kLmZm]) |
                               (cur & msk[i][kLmXin])) & q[i];
            cl[i] = cur;
            grown |= cur ^ own;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) wcl[lane + 64 * i] = cl[i];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (!__any(grown != 0u)) break;
    }
    // 4. both walkers flip the cluster: every dword read first, then every
    // write (a store to one walker's array could alias a later load from the
    // other's, so reads and writes in turn would each wait for the last)
    int size = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int I = lane + 64 * i;
        if (I >= NC || !cl[i]) continue;
        size += __popc(cl[i]);
        uint32_t va[2][C], vb[2][C];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const int w = (c * NC + I) * C + m;
                va[c][m] = sa[w];
                vb[c][m] = sb[w];
            }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const uint32_t f = B::spread4((cl[i] >> (c * L + 4 * m)) & B::dword_bits(m));
                const int w = (c * NC + I) * C + m;
                sa[w] = va[c][m] ^ f;
                sb[w] = vb[c][m] ^ f;
            }
    }
    size = wave_sum(size);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // 5. energies (Eq. 1): wa's from its new spins; the move keeps the sum
    // of the pair's energies (on a boundary bond of the cluster the two
    // walkers agree at the outer site and disagree at the inner one, so the
    // two bond terms cancel before and after), which gives wb's
    // one colour-0 dword per lane and pass (NC * C dwords spread evenly over
    // the lanes, rather than whole columns, which leave a part-filled pass)
    int ea = 0;
    for (int u = lane; u < NC * C; u += 64) {
        const int col = u / C, m = u - col * C;
        const uint32_t kbm = Col::field_dword(sa, s_j, 0, col, m, sa[spin_at<L, kColMajor>(0, col, m)]);
        const int nvalid = (G::TAIL != 0 && m == C - 1) ? G::TAIL : 4;
        ea += static_cast<int32_t>(kKbBias) * nvalid - static_cast<int32_t>(byte_sum(kbm & Col::valid(m)));
    }
    ea = wave_sum(ea);
    if (lane == 0) {
        const int32_t pair = s_E[wa] + s_E[wb];
        s_E[wa] = ea;
        s_E[wb] = pair - ea;
        *size_out = size;
    }
}

template <int L, bool JF>
__global__ __launch_bounds__(kIcmNW * 64) void k_pticm(PtIcmJob job, uint32_t k0, uint32_t k1)
{
    using G = Geo<L>;
    using Col = Column<L, JF, kColMajor, kColMajorOdd>;
    constexpr int NT = kIcmNW * 64;
    constexpr int JDW = G::jdw_odd(JF ? 2 : 1);
    constexpr int SDW = G::SPIN_DW;
    extern __shared__ uint32_t lds[];
    const int T = job.T, W = 2 * T;
    uint32_t *s_spin = lds;                                  // [W][SDW]
    uint32_t *s_j = s_spin + W * SDW;
    uint32_t *s_thr = s_j + JDW;                             // [T][64]
    int32_t *s_E = reinterpret_cast<int32_t *>(s_thr + T * kIcmThr);
    int32_t *s_pos = s_E + W;
    int32_t *s_who = s_pos + W;                              // [copy * T + slot]
    int32_t *s_sw = s_who + W;                               // [copy * (T-1) + k]
    int32_t *s_fl = s_sw + 2 * (T - 1);                      // [T] cluster size per slot, this step
    uint32_t *s_nz = reinterpret_cast<uint32_t *>(s_fl + T);  // [6][SDW] nonzero-coupling masks
    uint32_t *s_lm = s_nz + 6 * SDW;                         // [kLmN][NC] link masks as bits
    uint32_t *s_wcl = s_lm + kLmN * G::NC;                   // [kIcmNW][ROW] cluster rows
    uint32_t *s_thrx = s_wcl + kIcmNW * IcmBits<L>::ROW;     // [T-1][mx] exchange thresholds

    const int tid = static_cast<int>(threadIdx.x);
    const int lane = tid & 63, wave = tid >> 6;
    const int run = static_cast<int>(blockIdx.x);
    const uint32_t chain = job.run0 + static_cast<uint32_t>(run);
    int8_t *spins = job.spins + static_cast<int64_t>(run) * W * G::N;

    // ---- set-up ---------------------------------------------------------
    for (int w = tid; w < W * SDW; w += NT) s_spin[w] = 0u;
    for (int w = tid; w < T * kIcmThr; w += NT) {
        const int slot = w / kIcmThr, e = w - slot * kIcmThr;
        s_thr[w] = thr_entry(job.thr + slot * job.K, job.K, e);
    }
    if (tid < W) {
        s_E[tid] = 0;
        int p = job.init_random ? tid % T : job.pos[run * W + tid];
        if (p < 0 || p >= T) p = -1;   // out of range: not a permutation
        s_pos[tid] = p;
        s_who[tid] = -1;
    }
    if (tid < 2 * (T - 1)) s_sw[tid] = 0;
    for (int w = tid; w < (T - 1) * job.mx; w += NT) {
        const int k = w / job.mx, e = w - k * job.mx;
        s_thrx[w] = job.thrx[static_cast<int64_t>(k) * job.M + e];
    }
    load_couplings<L, JF, kColMajorOdd>(s_j, job.J, job.jenc, tid, NT);
    __syncthreads();
    if (tid < W && s_pos[tid] >= 0) s_who[(tid / T) * T + s_pos[tid]] = tid;
    // a copy whose pos is not a permutation of its slots leaves a slot
    // without a walker: the run then starts from the identity (every LDS
    // index stays in range)
    if (__syncthreads_or(tid < W && s_who[tid] < 0) && tid < W) {
        s_pos[tid] = tid % T;
        s_who[tid] = tid;
    }
    // the bonds a cluster grows along (nonzero couplings), per dword and
    // direction, for the whole run
    for (int w = tid; w < SDW; w += NT) {
        const int c = w / (G::NC * G::C), col = (w / G::C) % G::NC, m = w % G::C;
#pragma unroll
        for (int d = 0; d < 6; ++d) s_nz[d * SDW + w] = Col::nonzero_coupling(s_j, c, col, d, m);
    }
    if (tid < T) s_fl[tid] = 0;
    __syncthreads();
    // the same links as bits, per item (double column) and direction, in the
    // receiving site's frame, stored with the halves exchanged
    for (int it = tid; it < G::NC; it += NT) {
        using B = IcmBits<L>;
        const uint32_t even0 = Col::neighbours(0, it).even_x;   // colour-0 bytes whose x is even
        uint32_t lmk[kLmN] = {};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t ex = c ? ~even0 : even0;
#pragma unroll
            for (int m = 0; m < G::C; ++m) {
                const int w = (c * G::NC + it) * G::C + m;
                const int sh = c * L + 4 * m;
                const uint32_t keep = B::dword_bits(m);
                const uint32_t z0 = s_nz[w], z1 = s_nz[SDW + w];
                lmk[kLmZp] |= (B::gather4(s_nz[4 * SDW + w]) & keep) << sh;
                lmk[kLmZm] |= (B::gather4(s_nz[5 * SDW + w]) & keep) << sh;
                lmk[kLmXin] |= (B::gather4((z0 & ex) | (z1 & ~ex)) & keep) << sh;
                lmk[kLmXm] |= (B::gather4(z1 & ex) & keep) << sh;
                lmk[kLmXp] |= (B::gather4(z0 & ~ex) & keep) << sh;
                lmk[kLmYp] |= (B::gather4(s_nz[2 * SDW + w]) & keep) << sh;
                lmk[kLmYm] |= (B::gather4(s_nz[3 * SDW + w]) & keep) << sh;
            }
        }
#pragma unroll
        for (int d = 0; d < kLmN; ++d) s_lm[d * G::NC + it] = B::swap(lmk[d]);
    }
    {
        uint8_t *sb = reinterpret_cast<uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < W * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            load_spins_one<L>(sb + wk * SDW * 4, q, job.init_random != 0, spins + static_cast<int64_t>(wk) * G::N,
                              static_cast<uint32_t>(wk), chain, k0, k1);
        }
    }
    __syncthreads();
    for (int u = tid; u < W * G::NC; u += NT) {
        const int wk = u / G::NC;
        atomicAdd(&s_E[wk], Col::column_energy_of(s_spin + wk * SDW, s_j, u - wk * G::NC));
    }
    __syncthreads();

    // a lane's prepared sweep unit (when W * NC units fit the lanes)
    const bool prep = W * G::NC <= NT;
    const bool pact = tid < W * G::NC;
    const int pwk = pact ? tid / G::NC : 0;
    const typename Col::Unit pun =
        Col::make_unit(pact ? tid - pwk * G::NC : 0, static_cast<uint32_t>(pwk), chain, k0, k1);

    for (int ti = 0; ti < job.n_steps; ++ti) {
        const uint32_t t = static_cast<uint32_t>(job.step0 + ti);
        // ---- 1. sweeps ----------------------------------------------------------
        if (prep) {
            // one (walker, column) unit per lane, the same every step: its
            // neighbours and the step-independent Philox products are kept
            int32_t acc = 0;
            const uint32_t *tbl = s_thr + s_pos[pwk] * kIcmThr;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (pact)
                    acc += Col::template metropolis_unit<true>(s_spin + pwk * SDW, s_j, tbl, c, pun,
                                                               2u * t + static_cast<uint32_t>(c), k0, k1);
                if (c == 0) __syncthreads();
            }
            if (pact && acc != 0) atomicAdd(&s_E[pwk], acc);
            __syncthreads();
        } else for (int c = 0; c < 2; ++c) {
            for (int u = tid; u < W * G::NC; u += NT) {
                const int wk = u / G::NC;
                const int col = u - wk * G::NC;
                const int32_t dE = Col::template metropolis<true>(
                    s_spin + wk * SDW, s_j, s_thr + s_pos[wk] * kIcmThr, c, col, 2u * t + static_cast<uint32_t>(c),
                    static_cast<uint32_t>(wk), chain, k0, k1);
                if (dE != 0) atomicAdd(&s_E[wk], dE);
            }
            __syncthreads();
        }
        // ---- 2. cluster moves: slot k's by wave (k - icm_from) mod 12 ---------------
        for (int k = job.icm_from + wave; k < T; k += kIcmNW)
            icm_move_wave<L, JF>(s_spin, s_j, s_lm, s_wcl + wave * IcmBits<L>::ROW, s_who[k], s_who[T + k], k, t, chain, k0,
                                 k1, lane, s_E, s_fl + k);
        __syncthreads();
        // ---- 3. exchanges inside each copy ---------------------------------------
        if (tid < 2 * T) {
            const int cp = tid / T, k = tid - cp * T;
            if (k + 1 < T && ((k ^ static_cast<int>(t)) & 1) == 0) {
                // the word is drawn before the energies are read: it depends
                // on the counter alone
                const uint32_t ux = philox10(static_cast<uint32_t>(k + cp * T), t, 0xFFFFFFFFu, chain, k0, k1).w[0];
                const int a = s_who[cp * T + k], b = s_who[cp * T + k + 1];
                const int32_t D = s_E[a] - s_E[b];
                bool acc = D <= 0;
                if (!acc) {
                    const int32_t m = D / 2;
                    if (m <= job.mx)
                        acc = ux < s_thrx[k * job.mx + (m - 1)];
                    else
                        acc = (m <= job.M) && (ux < job.thrx[static_cast<int64_t>(k) * job.M + (m - 1)]);
                }
                if (acc) {
                    s_who[cp * T + k] = b;
                    s_who[cp * T + k + 1] = a;
                    s_pos[b] = k;
                    s_pos[a] = k + 1;
                    s_sw[cp * (T - 1) + k] += 1;
                }
            }
        }
        if (tid >= 64 && tid < 128) {
            int32_t e = 0x7FFFFFFF;
            for (int w = lane; w < W; w += 64) e = min(e, s_E[w]);
            e = __ockl_wfred_min_i32(e);
            if (lane == 0) {
                if (job.emin_trace) job.emin_trace[static_cast<int64_t>(run) * job.n_steps + ti] = e;
                if (job.icm_flipped) {
                    int32_t flipped = 0;
                    for (int k = job.icm_from; k < T; ++k) flipped += s_fl[k];
                    job.icm_flipped[static_cast<int64_t>(run) * job.n_steps + ti] = flipped;
                }
            }
        }
        __syncthreads();
    }

    // ---- write-back ---------------------------------------------------------
    {
        const uint8_t *sb = reinterpret_cast<const uint8_t *>(s_spin);
        constexpr int Q = G::N / 4;
        for (int w = tid; w < W * Q; w += NT) {
            const int wk = w / Q;
            const int q = w - wk * Q;
            store_spins_one<L>(sb + wk * SDW * 4, q, spins + static_cast<int64_t>(wk) * G::N);
        }
    }
    if (tid < W) {
        job.energy[run * W + tid] = s_E[tid];
        job.pos[run * W + tid] = s_pos[tid];
    }
    if (job.swap_acc && tid < 2 * (T - 1)) job.swap_acc[run * 2 * (T - 1) + tid] += static_cast<uint32_t>(s_sw[tid]);
}

template <int L>
static int launch_pticm(const PtIcmJob &job, int n_runs, uint32_t k0, uint32_t k1, hipStream_t stream)
{
    constexpr bool JF = false;   // E only in LDS: fewer coupling reads (as in PT)
    auto kern = k_pticm<L, JF>;
    const size_t kLds = lds_dynamic_cap(reinterpret_cast<const void *>(kern));
    const size_t base = pticm_lds_bytes<L, JF>(job.T, 0);
    if (base > kLds)
        return fail(SG_EUNSUPPORTED, "sg_pticm_run: L = %d with T = %d needs %zu bytes of LDS", L, job.T, base);
    // the exchange-table prefix held in LDS: up to kIcmMx entries per pair,
    // as many as the LDS left over allows (later entries are read from HBM)
    PtIcmJob jb = job;
    jb.mx = static_cast<int32_t>(std::min<size_t>({static_cast<size_t>(job.M), static_cast<size_t>(kIcmMx),
                                                   (kLds - base) / (4 * static_cast<size_t>(job.T - 1))}));
    const size_t bytes = pticm_lds_bytes<L, JF>(job.T, jb.mx);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_pticm_run: LDS attribute: %s", hipGetErrorString(err));
    (void)hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(n_runs), dim3(kIcmNW * 64), bytes, stream, jb, k0, k1);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_pticm_run: launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

}  // namespace sg

using namespace sg;

extern "C" int sg_pticm_run(const sg_instance *inst, const sg_pticm_args *args, const uint32_t *thr,
                            const uint32_t *thrx, int8_t *spins, int32_t *energy_out, int32_t *pos,
                            int32_t *emin_trace, uint32_t *swap_acc, int32_t *icm_flipped, void *stream)
{
    if (!inst || !args) return fail(SG_EINVAL, "sg_pticm_run: NULL instance or args");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "sg_pticm_run: L = %d must be even in [4, %d]", inst->L, SG_MAX_L);
    if (!inst->J && !inst->jenc) return fail(SG_EINVAL, "sg_pticm_run: instance has no couplings");
    if (!thr || !thrx || !spins || !energy_out || !pos) return fail(SG_EINVAL, "sg_pticm_run: NULL array");
    if (args->n_runs < 1 || args->n_steps < 1)
        return fail(SG_EINVAL, "sg_pticm_run: n_runs = %d, n_steps = %d", args->n_runs, args->n_steps);
    if (args->T < 2 || args->T > SG_PTICM_MAX_T)
        return fail(SG_EINVAL, "sg_pticm_run: T = %d outside [2, %d]", args->T, SG_PTICM_MAX_T);
    if (args->K < 1 || args->K > SG_K_MAX || args->M < 1)
        return fail(SG_EINVAL, "sg_pticm_run: K = %d, M = %d", args->K, args->M);
    if (args->icm_from < 0) return fail(SG_EINVAL, "sg_pticm_run: icm_from = %d", args->icm_from);
    if (args->step0 < 0 || static_cast<int64_t>(args->step0) + args->n_steps > (1 << 30))
        return fail(SG_ERANGE, "sg_pticm_run: steps must stay below 2^30");
    if (static_cast<uint64_t>(args->run0) + static_cast<uint64_t>(args->n_runs) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "sg_pticm_run: run counter words overflow");
    if ((reinterpret_cast<uintptr_t>(spins) & 3u) != 0) return fail(SG_EINVAL, "sg_pticm_run: spins must be 4-byte aligned");
    PtIcmJob job{};
    job.J = inst->J;
    job.jenc = inst->jenc;
    job.thr = thr;
    job.thrx = thrx;
    job.spins = spins;
    job.energy = energy_out;
    job.pos = pos;
    job.emin_trace = emin_trace;
    job.swap_acc = swap_acc;
    job.icm_flipped = icm_flipped;
    job.run0 = args->run0;
    job.T = args->T;
    job.n_steps = args->n_steps;
    job.step0 = args->step0;
    job.K = args->K;
    job.M = args->M;
    job.icm_from = args->icm_from;
    job.init_random = args->init_random ? 1 : 0;
    clear_error();
    const uint32_t k0 = static_cast<uint32_t>(args->seed), k1 = static_cast<uint32_t>(args->seed >> 32);
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (inst->L) {
    case 4: return launch_pticm<4>(job, args->n_runs, k0, k1, st);
    case 6: return launch_pticm<6>(job, args->n_runs, k0, k1, st);
    case 8: return launch_pticm<8>(job, args->n_runs, k0, k1, st);
    case 10: return launch_pticm<10>(job, args->n_runs, k0, k1, st);
    case 12: return launch_pticm<12>(job, args->n_runs, k0, k1, st);
    case 14: return launch_pticm<14>(job, args->n_runs, k0, k1, st);
    case 16: return launch_pticm<16>(job, args->n_runs, k0, k1, st);
    default: return fail(SG_EUNSUPPORTED, "sg_pticm_run: L = %d is above the LDS-resident range", inst->L);
    }
}
