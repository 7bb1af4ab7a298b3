// pticm.hip -- parallel tempering with isoenergetic cluster moves (App. D,
// PT+ICM; the cluster move is Houdayer's two-replica move as combined with
// PT by Zhu, Ochoa and Katzgraber) and its C-ABI entry point.
//
// One work group runs one run: two copies of a T-slot ladder (2T walkers),
// all LDS-resident in the colour-split column layout.  A step is the sweep
// of every walker, then for every slot k >= icm_from one cluster move
// between the two walkers at slot k, then the even/odd exchanges inside
// each copy.  A cluster move works on byte masks in the same layout as the
// spins: the disagreement mask is the XOR of the two walkers, a block-wide
// prefix count picks the seed, and the cluster grows by repeated expansion
// through neighbouring disagreeing sites joined by nonzero couplings (the
// same byte shuffles as the local fields) until a pass adds nothing; both
// walkers then XOR the cluster in.
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
    int32_t G;              // slots whose cluster moves run together
};

constexpr int kIcmNW = 12;          // 768 lanes per run
constexpr int kIcmThr = kThrEntries;

// LDS of one run with cluster moves of ng slots at once
template <int L, bool JF>
constexpr size_t pticm_lds_bytes(int T, int ng)
{
    using G = Geo<L>;
    const size_t W = 2 * static_cast<size_t>(T);
    return (W * G::SPIN_DW + G::jdw_odd(JF ? 2 : 1) + static_cast<size_t>(T) * kIcmThr + 3 * W +
            2 * (static_cast<size_t>(T) - 1) + 2 * static_cast<size_t>(ng) * G::SPIN_DW + 64 +
            2 * static_cast<size_t>(T) + 6 * static_cast<size_t>(G::SPIN_DW)) * 4;
}

// One growth pass over the double column `col` of one slot's cluster: both
// colour columns of index col, i.e. the sites with x in {2k, 2k+1} at one
// y, every z.  Its z-links and half of its x-links stay inside it.  The
// pass reads the cluster bits of the four neighbouring double columns
// once, then adds, until nothing changes, every disagreeing site (q) joined
// by a nonzero coupling (nz: [6][SPIN_DW] masks) to a cluster site, inside
// the item or in those neighbours.  cl is the cluster, laid out like q.
// Returns 1 if anything was added.  Bits other lanes add meanwhile are seen
// by a later pass, so the fixpoint of the passes is the connected component
// of the seed, whatever the order.
template <int L, bool JF>
__device__ int icm_grow_column(const uint32_t *q, uint32_t *cl, const uint32_t *nz, int col)
{
    using G = Geo<L>;
    using Col = Column<L, JF, kColMajor, kColMajorOdd>;
    constexpr int C = G::C, NC = G::NC, SDW = G::SPIN_DW;
    uint32_t qq[2][C], cc[2][C];
    uint32_t open = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < C; ++m) {
            qq[c][m] = q[(c * NC + col) * C + m];
            cc[c][m] = cl[(c * NC + col) * C + m];
            open |= qq[c][m] & ~cc[c][m];
        }
    if (!open) return 0;   // every disagreeing site here is in already
    const typename Col::Nbr n = Col::neighbours(0, col);
    // first what the neighbouring double columns reach (added at once);
    // ix, nzp, nzm: the nonzero-coupling masks of the links inside the item
    // (x, +z, -z)
    uint32_t ix[2][C], nzp[2][C], nzm[2][C];
    uint32_t first = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint32_t ex = c ? ~n.even_x : n.even_x;   // bytes whose x is even
        const int oc = c ^ 1;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int w = (c * NC + col) * C + m;
            const uint32_t xp = cl[(oc * NC + n.xp) * C + m], xm = cl[(oc * NC + n.xm) * C + m];
            const uint32_t yp = cl[(oc * NC + n.yp) * C + m], ym = cl[(oc * NC + n.ym) * C + m];
            const uint32_t z0 = nz[w], z1 = nz[SDW + w];
            const uint32_t nw = ((xp & ~ex & z0) | (xm & ex & z1) | (yp & nz[2 * SDW + w]) | (ym & nz[3 * SDW + w])) &
                                qq[c][m] & ~cc[c][m];
            cc[c][m] |= nw;
            first |= nw;
            ix[c][m] = (z0 & ex) | (z1 & ~ex);
            nzp[c][m] = nz[4 * SDW + w];
            nzm[c][m] = nz[5 * SDW + w];
        }
    }
    int added = first != 0;
    for (;;) {   // ends: every round adds a site or stops
        uint32_t ch = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t(&S)[C] = cc[c ^ 1];
#pragma unroll
            for (int m = 0; m < C; ++m) {
                uint32_t zp, zm;
                if (G::TAIL != 0 && m == C - 1)
                    zp = __builtin_amdgcn_perm(S[0], S[C - 1], 0x00000401u);
                else
                    zp = __builtin_amdgcn_alignbyte(S[(m + 1) % C], S[m], 1);
                if (G::TAIL != 0 && m == 0)
                    zm = __builtin_amdgcn_perm(S[0], S[C - 1], 0x06050401u);
                else
                    zm = __builtin_amdgcn_alignbyte(S[m], S[(m + C - 1) % C], 3);
                const uint32_t reach = (S[m] & ix[c][m]) | (zp & nzp[c][m]) | (zm & nzm[c][m]);
                const uint32_t nw = reach & qq[c][m] & ~cc[c][m];
                cc[c][m] |= nw;
                ch |= nw;
            }
        }
        if (!ch) break;
        added = 1;
    }
    if (added)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int m = 0; m < C; ++m) cl[(c * NC + col) * C + m] = cc[c][m];
    return added;
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
    uint32_t *s_q = reinterpret_cast<uint32_t *>(s_sw + 2 * (T - 1));   // disagreement masks [G][SDW]
    uint32_t *s_cl = s_q + job.G * SDW;                      // cluster masks [G][SDW]
    int32_t *s_misc = reinterpret_cast<int32_t *>(s_cl + job.G * SDW);   // 64 words: scan, flip counts
    int32_t *s_n = s_misc + 64;                              // [G] disagreeing sites per slot
    int32_t *s_tgt = s_n + T;                                // [G] seed position per slot
    uint32_t *s_nz = reinterpret_cast<uint32_t *>(s_tgt + T);  // [6][SDW] nonzero-coupling masks

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

    for (int ti = 0; ti < job.n_steps; ++ti) {
        const uint32_t t = static_cast<uint32_t>(job.step0 + ti);
        // ---- 1. sweeps ----------------------------------------------------------
        for (int c = 0; c < 2; ++c) {
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
        // ---- 2. cluster moves: the slots icm_from.. in groups of G at once -------
        // (the slots' walker pairs are disjoint, so the moves are independent).
        // Element p = g * SDW + w is dword w of slot k0s + g; each lane owns a
        // contiguous range of elements, so a block scan over the lanes orders
        // the disagreeing sites slot by slot, then by (colour, column, height).
        int32_t flipped = 0;
        for (int k0s = job.icm_from; k0s < T; k0s += job.G) {
            const int gn = min(job.G, T - k0s);
            const int tot = gn * SDW;
            const int per = (tot + NT - 1) / NT;
            const int p0 = min(tid * per, tot), p1 = min(p0 + per, tot);
            if (tid < gn) s_n[tid] = 0;
            __syncthreads();
            int lsum = 0;
            for (int p = p0; p < p1; ++p) {
                const int g = p / SDW, w = p - g * SDW;
                const uint32_t q = s_spin[s_who[k0s + g] * SDW + w] ^ s_spin[s_who[T + k0s + g] * SDW + w];
                s_q[p] = q;
                s_cl[p] = 0u;
                const int cnt = __popc(q) >> 3;
                if (cnt) atomicAdd(&s_n[g], cnt);
                lsum += cnt;
            }
            int incl = lsum;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            if (lane == 63) s_misc[wave] = incl;
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int w = 0; w < kIcmNW; ++w) {
                    const int v = s_misc[w];
                    s_misc[w] = acc;
                    acc += v;
                }
            }
            if (tid < gn) {
                // seed of slot k0s + tid: its position among all disagreeing
                // sites of the group (-1: the two walkers agree everywhere)
                int start = 0;
                for (int g = 0; g < tid; ++g) start += s_n[g];
                const int n = s_n[tid];
                int tgt = -1;
                if (n > 0) {
                    const Rand4 uu = philox10(static_cast<uint32_t>(k0s + tid), t, 0xFFFFFFFEu, chain, k0, k1);
                    tgt = start + static_cast<int>((static_cast<uint64_t>(uu.w[0]) * static_cast<uint64_t>(n)) >> 32);
                }
                s_tgt[tid] = tgt;
            }
            __syncthreads();
            {
                const int excl = s_misc[wave] + incl - lsum;
                for (int g = 0; g < gn; ++g) {
                    const int tgt = s_tgt[g];
                    if (tgt < excl || tgt >= excl + lsum) continue;
                    int r = tgt - excl;
                    for (int p = p0; p < p1; ++p) {
                        const uint32_t q = s_q[p];
                        const int cnt = __popc(q) >> 3;
                        if (r >= cnt) {
                            r -= cnt;
                            continue;
                        }
                        for (int b2 = 0; b2 < 4; ++b2)
                            if ((q >> (8 * b2)) & 0xFFu) {
                                if (r == 0) {
                                    s_cl[p] = 0xFFu << (8 * b2);
                                    break;
                                }
                                --r;
                            }
                        break;
                    }
                }
            }
            __syncthreads();
            // growth of every slot's cluster until a pass adds nothing; a
            // work item is one double column of one slot (icm_grow_column)
            int grown = 1;
            while (grown) {
                int add = 0;
                for (int it = tid; it < gn * G::NC; it += NT) {
                    const int g = it / G::NC;
                    add |= icm_grow_column<L, JF>(s_q + g * SDW, s_cl + g * SDW, s_nz, it - g * G::NC);
                }
                grown = __syncthreads_or(add);
            }
            // flip every cluster in both walkers of its slot
            int fl = 0;
            for (int p = p0; p < p1; ++p) {
                const int g = p / SDW, w = p - g * SDW;
                const uint32_t cl = s_cl[p];
                if (!cl) continue;
                s_spin[s_who[k0s + g] * SDW + w] ^= cl;
                s_spin[s_who[T + k0s + g] * SDW + w] ^= cl;
                fl += __popc(cl) >> 3;
            }
            for (int off = 32; off > 0; off >>= 1) fl += __shfl_xor(fl, off, 64);
            if (lane == 0) s_misc[32 + wave] = fl;
            if (tid < 2 * gn) s_E[s_who[(tid / gn) * T + k0s + tid % gn]] = 0;
            __syncthreads();
            // energies of the moved walkers
            for (int u = tid; u < 2 * gn * G::NC; u += NT) {
                const int pw = u / G::NC;
                const int wk = s_who[(pw / gn) * T + k0s + pw % gn];
                atomicAdd(&s_E[wk], Col::column_energy_of(s_spin + wk * SDW, s_j, u - pw * G::NC));
            }
            if (tid == 0) {
                int tot_fl = 0;
                for (int w = 0; w < kIcmNW; ++w) tot_fl += s_misc[32 + w];
                s_misc[kIcmNW + 2] = tot_fl;
            }
            __syncthreads();
            flipped += s_misc[kIcmNW + 2];
            __syncthreads();
        }
        // ---- 3. exchanges inside each copy ---------------------------------------
        if (tid < 2 * T) {
            const int cp = tid / T, k = tid - cp * T;
            if (k + 1 < T && ((k ^ static_cast<int>(t)) & 1) == 0) {
                const int a = s_who[cp * T + k], b = s_who[cp * T + k + 1];
                const int32_t D = s_E[a] - s_E[b];
                bool acc = D <= 0;
                if (!acc) {
                    const int32_t m = D / 2;
                    const Rand4 u = philox10(static_cast<uint32_t>(k + cp * T), t, 0xFFFFFFFFu, chain, k0, k1);
                    acc = (m <= job.M) && (u.w[0] < job.thrx[static_cast<int64_t>(k) * job.M + (m - 1)]);
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
            for (int off = 32; off > 0; off >>= 1) e = min(e, __shfl_xor(e, off, 64));
            if (lane == 0) {
                if (job.emin_trace) job.emin_trace[static_cast<int64_t>(run) * job.n_steps + ti] = e;
                if (job.icm_flipped) job.icm_flipped[static_cast<int64_t>(run) * job.n_steps + ti] = flipped;
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
    constexpr size_t kLds = 160 * 1024;
    const size_t base = pticm_lds_bytes<L, JF>(job.T, 1);
    if (base > kLds)
        return fail(SG_EUNSUPPORTED, "sg_pticm_run: L = %d with T = %d needs %zu bytes of LDS", L, job.T, base);
    // as many slots' cluster moves at once as the LDS left over holds
    PtIcmJob jb = job;
    const int slots = std::max(1, job.T - job.icm_from);
    const size_t per_slot = 2 * static_cast<size_t>(Geo<L>::SPIN_DW) * 4;
    jb.G = static_cast<int32_t>(std::min<size_t>(slots, 1 + (kLds - base) / per_slot));
    const size_t bytes = pticm_lds_bytes<L, JF>(job.T, jb.G);
    auto kern = k_pticm<L, JF>;
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
