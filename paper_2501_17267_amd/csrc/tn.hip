// tn.hip -- tensor-network fragment decimation (Sec. I, App. A-C) on the
// device: exact contraction of every fragment's free spins, one table per
// (site, value of the site), phase by phase.
//
// LDS tier: one work group holds a table of up to 2^lds_bits doubles (or
// int32 for the tropical form) and runs the whole elimination program of
// its shape, one block barrier per eliminated spin.
// Workspace tier: larger tables live in the caller's workspace; every
// round (one elimination step, or two fused, see TnRound) is one launch over
// all tables of a batch that updates only the canonical entries of its table
// (see TnStep), up to kTnPairsPerThread read assignments per thread.
// A sum-product table is renormalised after every round by the power of two
// that brings its largest entry into [1, 2) (exact scaling, the exponents
// summed beside it).  With |h| <= kTnHMax no product overflows for
// beta <= 14 when every step is a round, and for beta <= 9.5 with fused
// rounds (raw values below 8 exp(2 kTnHMax beta) before a round's scale).
// A decision kernel per phase turns the two results of each site into its
// spin and score.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "tn.hpp"
#include "variants.hpp"

namespace sg {

namespace {

constexpr int kTnHMax = 24;                  // |h_v| <= 6 * 4
constexpr int kTnWeights = 2 * kTnHMax + 1;  // exp(-beta k), k = -24..24
constexpr double kLn2 = 0.69314718055994530942;

struct TnWeights {
    double w[kTnWeights];
};

struct TnJob {
    const int8_t *J;       // [n_inst][6][N]
    int8_t *dec;           // [n_inst][N]
    double *score;         // [n_inst][N] or null
    const TnShape *shapes;
    const TnStep *steps;
    const TnRound *rounds;
    const TnItem *items;
    double *res;           // [n_inst][items of the phase][2]
    int32_t L, h, l;
    int64_t N;
    double beta;
    int32_t fuse;          // 1: the plan's rounds, 0: one step per round
};

// the eliminated spin's slot, its active neighbours' slots and couplings, and
// the field from fixed and centre neighbours
struct TnDesc {
    uint32_t slots;        // 5 bits per direction
    int8_t J[6];           // 0 where the neighbour is not active
    int16_t hc;
    int32_t a;
};

__device__ inline int64_t tn_wrap_site(const TnJob &jb, int64_t site, int dx, int dy, int dz)
{
    const int L = jb.L;
    const int x = static_cast<int>(site % L), y = static_cast<int>((site / L) % L),
              z = static_cast<int>(site / (static_cast<int64_t>(L) * L));
    const int gx = (x + dx + L) % L, gy = (y + dy + L) % L, gz = (z + dz + L) % L;
    return gx + static_cast<int64_t>(L) * (gy + static_cast<int64_t>(L) * gz);
}

// global index of local fragment site j of the fragment centred on `site`
__device__ inline int64_t tn_local_site(const TnJob &jb, int64_t site, int j)
{
    const int l = jb.l;
    return tn_wrap_site(jb, site, j % l - jb.h, (j / l) % l - jb.h, j / (l * l) - jb.h);
}

__device__ inline int64_t tn_nbr(const TnJob &jb, int64_t g, int d)
{
    return tn_wrap_site(jb, g, (d == 0) - (d == 1), (d == 2) - (d == 3), (d == 4) - (d == 5));
}

__device__ inline TnDesc tn_desc(const TnJob &jb, const int8_t *J, const int8_t *dec, int64_t site, int sc,
                                 const TnStep &st)
{
    TnDesc D{};
    const int64_t g = tn_local_site(jb, site, st.lv);
    int hc = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int code = st.code[d];
        if (code == kTnNone) continue;
        const int Jd = J[d * jb.N + g];
        if (code >= 0) {
            D.J[d] = static_cast<int8_t>(Jd);
            D.slots |= static_cast<uint32_t>(code) << (5 * d);
        } else if (code == kTnConst) {
            hc += Jd * dec[tn_nbr(jb, g, d)];
        } else {
            hc += Jd * sc;
        }
    }
    D.hc = static_cast<int16_t>(hc);
    D.a = st.a;
    return D;
}

// energy of the centre's bonds to fixed fragment sites, at centre value sc
__device__ inline int tn_centre_energy(const TnJob &jb, const int8_t *J, const int8_t *dec, int64_t site, int sc,
                                       const TnShape &sh)
{
    int e = 0;
    for (int d = 0; d < 6; ++d)
        if (sh.ccode[d] == kTnConst) e += J[d * jb.N + site] * dec[tn_nbr(jb, site, d)];
    return e * sc;
}

// field without the clamp (the canonical-slot part of a split field)
__device__ inline int tn_field_raw(const TnDesc &D, uint32_t I0)
{
    int hh = D.hc;
#pragma unroll
    for (int d = 0; d < 6; ++d) hh += D.J[d] * (1 - 2 * static_cast<int>((I0 >> ((D.slots >> (5 * d)) & 31u)) & 1u));
    return hh;
}

__device__ inline int tn_field(const TnDesc &D, uint32_t I0)
{
    int hh = D.hc;
#pragma unroll
    for (int d = 0; d < 6; ++d) hh += D.J[d] * (1 - 2 * static_cast<int>((I0 >> ((D.slots >> (5 * d)) & 31u)) & 1u));
    // |h| <= 24 for couplings in [-4, 4]; the clamp only keeps the weight
    // lookup inside its table for invalid couplings
    return min(max(hh, -kTnHMax), kTnHMax);
}

__device__ inline uint32_t tn_pair_index(uint32_t p, int a)
{
    const uint32_t low = (1u << a) - 1u;
    return ((p >> a) << (a + 1)) | (p & low);
}

// (T0 w(+1) + T1 w(-1)) scale with both products rounded before the sum (no
// fused multiply-add): a table and
// its mirror image (every spin flipped) then give bit-identical results, so
// a site whose fragment has no fixed coupling scores exactly 0
__device__ inline double tn_pair_sum(double t0, double w0, double t1, double w1, double scale)
{
#pragma clang fp contract(off)
    const double p0 = t0 * w0;
    const double p1 = t1 * w1;
    return (p0 + p1) * scale;
}

// ln Z of a finished table: ln T + (applied exponents) ln 2 - beta E_centre
__device__ inline double tn_log_result(double t, int64_t e_sum, double beta, int es)
{
#pragma clang fp contract(off)
    const double a = log(t);
    const double b = static_cast<double>(e_sum) * kLn2;
    const double c = beta * static_cast<double>(es);
    return (a + b) - c;
}

__device__ inline int wave_max_int(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// ---- LDS tier ---------------------------------------------------------------

template <bool TROP>
__global__ __launch_bounds__(kTnThreads) void k_tn_lds(TnJob jb, TnWeights wt, int item0, int n_items_q, int n_lds,
                                                        int tab_bytes, int desc_steps)
{
    using T = typename std::conditional<TROP, int32_t, double>::type;
    extern __shared__ __align__(16) char smem[];
    T *tab = reinterpret_cast<T *>(smem);
    TnDesc *desc = reinterpret_cast<TnDesc *>(smem + tab_bytes);
    double *w = reinterpret_cast<double *>(desc + desc_steps);
    int *s_emax = reinterpret_cast<int *>(w + kTnWeights);   // [2][waves]

    const int tid = static_cast<int>(threadIdx.x);
    const int gid = static_cast<int>(blockIdx.x);
    const int cv = gid & 1;
    const int k = (gid >> 1) % n_lds;
    const int inst = (gid >> 1) / n_lds;
    const int sc = cv ? -1 : 1;
    const TnItem it = jb.items[item0 + k];
    const TnShape sh = jb.shapes[it.shape];
    const int8_t *J = jb.J + static_cast<int64_t>(inst) * 6 * jb.N;
    const int8_t *dec = jb.dec + static_cast<int64_t>(inst) * jb.N;
    const int W = sh.W, ns = sh.n_steps;

    for (int t = tid; t < ns; t += kTnThreads) desc[t] = tn_desc(jb, J, dec, it.site, sc, jb.steps[sh.step0 + t]);
    if (!TROP)
        for (int i = tid; i < kTnWeights; i += kTnThreads) w[i] = wt.w[i];
    for (int i = tid; i < (1 << W); i += kTnThreads) tab[i] = TROP ? T(0) : T(1);
    __syncthreads();

    const int half = W > 0 ? 1 << (W - 1) : 0;
    double scale = 1.0;
    int e_prev = 0, e_sum = 0;
    // renormalised after every round, as the workspace tier is
    const int nr = jb.fuse ? sh.n_rounds : ns;
    for (int r = 0; r < nr; ++r) {
        int t0 = r, n_sub = 1;
        if (jb.fuse) {
            const TnRound R = jb.rounds[sh.round0 + r];
            t0 = R.step;
            n_sub = 1 + R.fused;
        }
        if (!TROP && r > 0) {
            e_sum += e_prev;
            scale = ldexp(1.0, -e_prev);
        }
        double m = 0.0;
        if (n_sub == 1) {
            const TnDesc D = desc[t0];
            const uint32_t abit = 1u << D.a;
            for (int p = tid; p < half; p += kTnThreads) {
                const uint32_t I0 = tn_pair_index(static_cast<uint32_t>(p), D.a), I1 = I0 | abit;
                const int hh = tn_field(D, I0);
                T v;
                if (TROP) {
                    v = min(tab[I0] + hh, tab[I1] - hh);
                } else {
                    v = tn_pair_sum(tab[I0], w[kTnHMax + hh], tab[I1], w[kTnHMax - hh], scale);
                    m = fmax(m, static_cast<double>(v));
                }
                tab[I0] = v;
                tab[I1] = v;
            }
        } else {
            // a fused pair in one pass: each thread takes the four entries at
            // slots a, b = 0, 1 of an index, applies the first step to both
            // pairs along a and the second to the pair along b (the same
            // operations as two passes, without the barrier between them)
            const TnDesc D0 = desc[t0], D1 = desc[t0 + 1];
            const uint32_t abit = 1u << D0.a, bbit = 1u << D1.a;
            const int lo = min(D0.a, D1.a), hi = max(D0.a, D1.a);
            for (int p = tid; p < (half >> 1); p += kTnThreads) {
                const uint32_t I = tn_pair_index(tn_pair_index(static_cast<uint32_t>(p), lo), hi);
                const T e00 = tab[I], e10 = tab[I | abit], e01 = tab[I | bbit], e11 = tab[I | abit | bbit];
                const int h0 = tn_field(D0, I), h1 = tn_field(D0, I | bbit);
                const int g0 = tn_field(D1, I), g1 = tn_field(D1, I | abit);
                T u0, u1;
                if (TROP) {
                    const T v0 = min(e00 + h0, e10 - h0), v1 = min(e01 + h1, e11 - h1);
                    u0 = min(v0 + g0, v1 - g0);
                    u1 = min(v0 + g1, v1 - g1);
                } else {
                    const T v0 = tn_pair_sum(e00, w[kTnHMax + h0], e10, w[kTnHMax - h0], scale);
                    const T v1 = tn_pair_sum(e01, w[kTnHMax + h1], e11, w[kTnHMax - h1], scale);
                    u0 = tn_pair_sum(v0, w[kTnHMax + g0], v1, w[kTnHMax - g0], 1.0);
                    u1 = tn_pair_sum(v0, w[kTnHMax + g1], v1, w[kTnHMax - g1], 1.0);
                    m = fmax(m, fmax(static_cast<double>(u0), static_cast<double>(u1)));
                }
                tab[I] = u0;
                tab[I | bbit] = u0;
                tab[I | abit] = u1;
                tab[I | abit | bbit] = u1;
            }
        }
        if (!TROP) {
            const int e = wave_max_int(m > 0.0 ? ilogb(m) : INT_MIN);
            if ((tid & 63) == 0) s_emax[(r & 1) * (kTnThreads / 64) + (tid >> 6)] = e;
        }
        __syncthreads();
        if (!TROP) {
            int e = INT_MIN;
            for (int i = 0; i < kTnThreads / 64; ++i) e = max(e, s_emax[(r & 1) * (kTnThreads / 64) + i]);
            e_prev = e;
        }
    }
    if (tid == 0) {
        const int es = tn_centre_energy(jb, J, dec, it.site, sc, sh);
        double r;
        if (TROP)
            r = static_cast<double>(static_cast<int64_t>(tab[0]) + es);
        else
            r = tn_log_result(static_cast<double>(tab[0]), e_sum, jb.beta, es);
        jb.res[(static_cast<int64_t>(inst) * n_items_q + k) * 2 + cv] = r;
    }
}

// ---- workspace tier ----------------------------------------------------------

// a batch: instances [b0, b0 + nb), workspace items [k0, k1) of one phase
// (indices relative to the phase's first workspace item); its tables are
// numbered tix = ((instance - b0) (k1 - k0) + (item - k0)) 2 + (centre value)
struct TnBatch {
    int32_t item_hbm0;          // index in items of the phase's first workspace item
    int32_t res_k0;             // position of that item among the phase's items
    int32_t n_items_q;
    int32_t k0, k1, b0, nb;
    int32_t steps;              // row length of desc and emax (rounds <= steps)
    const int64_t *entry_pre;   // the phase's segment of the table-entry prefix
    int64_t ents_per_inst;
    struct TnTab *tabs;         // [tables]
    struct TnDescX *desc;       // [tables][rounds]
    int32_t *blkpre;            // [rounds][k1 - k0 + 1]: work groups of the items before
                                //   (one table; every instance and value has the same)
    int32_t *emax;              // [tables][rounds]
    int32_t *es;                // [tables]
    void *tables;
};

struct TnTab {
    int32_t n_rounds, W;
    int64_t off;                // first entry of the table in the batch's table region
};

// one round of one workspace table, ready to use: the field terms of the
// eliminated spin and the canonical bookkeeping of its first step (TnStep),
// and for a fused round the second step's field terms, new slots and the
// case of its slot b (TnRound)
struct __align__(16) TnDescX {
    TnDesc d;
    uint32_t newmask;
    uint8_t a_active, n_runs, n_base, fused;
    uint8_t run_start[8];
    uint8_t run_len[8];
    TnDesc d1;
    uint32_t newmask1;
    uint8_t b_mode, b_rank, read_bits, pad;
};
static_assert(sizeof(TnDescX) == 64, "TnDescX layout");

// the round r of a shape: its first step and whether it is fused
__device__ __host__ inline TnRound tn_round(const TnRound *rounds, const TnStep *steps, const TnShape &sh, int r,
                                            bool fuse)
{
    if (fuse) return rounds[sh.round0 + r];
    TnRound R{};
    R.step = static_cast<int16_t>(r);
    R.read_bits = steps[sh.step0 + r].n_base;
    return R;
}

// per (table, round): the round's descriptor; per table: its header, the
// centre's fixed-bond energy, and the exponent slots cleared
__global__ void k_tn_hbm_prep(TnJob jb, TnBatch bt)
{
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int nk = bt.k1 - bt.k0;
    const int64_t nt = static_cast<int64_t>(bt.nb) * nk * 2;
    if (gid >= nt * bt.steps) return;
    const int64_t tix = gid / bt.steps;
    const int t = static_cast<int>(gid - tix * bt.steps);
    const int cv = static_cast<int>(tix & 1);
    const int k = bt.k0 + static_cast<int>((tix >> 1) % nk);
    const int bi = static_cast<int>((tix >> 1) / nk);
    const int inst = bt.b0 + bi;
    const TnItem it = jb.items[bt.item_hbm0 + k];
    const TnShape sh = jb.shapes[it.shape];
    const int8_t *J = jb.J + static_cast<int64_t>(inst) * 6 * jb.N;
    const int8_t *dec = jb.dec + static_cast<int64_t>(inst) * jb.N;
    bt.emax[gid] = INT_MIN;
    if (t == 0) {
        TnTab tb;
        tb.n_rounds = jb.fuse ? sh.n_rounds : sh.n_steps;
        tb.W = sh.W;
        tb.off = static_cast<int64_t>(bi) * bt.ents_per_inst + (bt.entry_pre[k] - bt.entry_pre[bt.k0]) +
                 (static_cast<int64_t>(cv) << sh.W);
        bt.tabs[tix] = tb;
        bt.es[tix] = tn_centre_energy(jb, J, dec, it.site, cv ? -1 : 1, sh);
    }
    if (t < (jb.fuse ? sh.n_rounds : sh.n_steps)) {
        const TnRound R = tn_round(jb.rounds, jb.steps, sh, t, jb.fuse);
        const TnStep st = jb.steps[sh.step0 + R.step];
        TnDescX x{};
        x.d = tn_desc(jb, J, dec, it.site, cv ? -1 : 1, st);
        x.newmask = st.newmask;
        x.a_active = st.a_active;
        x.n_runs = st.n_runs;
        x.n_base = st.n_base;
        for (int r = 0; r < 8; ++r) {
            x.run_start[r] = st.run_start[r];
            x.run_len[r] = st.run_len[r];
        }
        x.fused = R.fused;
        x.read_bits = R.read_bits;
        if (R.fused) {
            const TnStep s1 = jb.steps[sh.step0 + R.step + 1];
            x.d1 = tn_desc(jb, J, dec, it.site, cv ? -1 : 1, s1);
            x.newmask1 = s1.newmask;
            x.b_mode = R.b_mode;
            x.b_rank = R.b_rank;
        }
        bt.desc[gid] = x;
    }
}

// per round: the prefix over the batch's items of their work groups
// (tn_table_blocks of the round's canonical reads; none once an item is done)
__global__ void k_tn_hbm_blocks(TnJob jb, TnBatch bt)
{
    const int t = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= bt.steps) return;
    const int nk = bt.k1 - bt.k0;
    constexpr int per = kTnThreads * kTnPairsPerThread;
    int32_t acc = 0;
    for (int kk = 0; kk < nk; ++kk) {
        bt.blkpre[t * (nk + 1) + kk] = acc;
        const TnShape sh = jb.shapes[jb.items[bt.item_hbm0 + bt.k0 + kk].shape];
        if (t < (jb.fuse ? sh.n_rounds : sh.n_steps))
            acc += ((1 << tn_round(jb.rounds, jb.steps, sh, t, jb.fuse).read_bits) + per - 1) / per;
    }
    bt.blkpre[t * (nk + 1) + nk] = acc;
}

// canonical index of read item p: the bits of p deposited into the step's runs
__device__ inline uint32_t tn_deposit(uint32_t p, const TnDescX &x)
{
    // the runs as two packed words (shifts rather than indexed bytes)
    uint64_t starts, lens;
    __builtin_memcpy(&starts, x.run_start, 8);
    __builtin_memcpy(&lens, x.run_len, 8);
    uint32_t I = 0;
    int used = 0;
    for (int r = 0; r < x.n_runs; ++r) {
        const int len = static_cast<int>((lens >> (8 * r)) & 0xFFu);
        I |= ((p >> used) & ((1u << len) - 1u)) << static_cast<int>((starts >> (8 * r)) & 0xFFu);
        used += len;
    }
    return I;
}

// the bits of v at the set bits of mask, packed from bit 0 in increasing order
__device__ inline uint32_t tn_extract(uint32_t v, uint32_t mask)
{
    uint32_t r = 0;
    int k = 0;
    for (uint32_t b = mask; b; b &= b - 1) r |= ((v >> __builtin_ctz(b)) & 1u) << k++;
    return r;
}

// round t of every table of the batch that has one: blocks_t work groups per
// (instance, centre value), each item's share given by the prefix blkpre[t]
template <bool TROP>
__global__ __launch_bounds__(kTnThreads) void k_tn_hbm_step(TnBatch bt, TnWeights wt, int t, int blocks_t)
{
    using T = typename std::conditional<TROP, int32_t, double>::type;
    __shared__ double w[kTnWeights];
    __shared__ int s_emax[kTnThreads / 64];
    __shared__ int32_t pre[kTnThreads + 1];
    __shared__ int32_t s_hn[64];   // field from the new slots, per combination
    __shared__ T s_v[kTnFuseMax][kTnThreads];   // a fused round's values between its steps
    const int tid = static_cast<int>(threadIdx.x);
    const int nk = bt.k1 - bt.k0;
    const int64_t g = static_cast<int64_t>(blockIdx.x) / blocks_t;   // (instance, value)
    const int rb = static_cast<int>(static_cast<int64_t>(blockIdx.x) - g * blocks_t);
    // the round's prefix row, staged in LDS (batches have at most kTnThreads items)
    const int32_t *row = bt.blkpre + static_cast<int64_t>(t) * (nk + 1);
    for (int i = tid; i <= nk; i += kTnThreads) pre[i] = row[i];
    if (!TROP)
        for (int i = tid; i < kTnWeights; i += kTnThreads) w[i] = wt.w[i];
    __syncthreads();
    int lo = 0, hi = nk - 1;   // the item: last kk with pre[kk] <= rb
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= rb)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int bpt = pre[lo + 1] - pre[lo];
    const int64_t tblk = rb - pre[lo];
    const int64_t tix = ((g >> 1) * nk + lo) * 2 + (g & 1);
    const TnTab tb = bt.tabs[tix];
    const TnDescX x = bt.desc[tix * bt.steps + t];
    T *tab = reinterpret_cast<T *>(bt.tables) + tb.off;
    const double scale = (!TROP && t > 0) ? ldexp(1.0, -bt.emax[tix * bt.steps + t - 1]) : 1.0;
    const int64_t items = int64_t{1} << x.read_bits;
    const int64_t stride = static_cast<int64_t>(bpt) * kTnThreads;
    const uint32_t abit = 1u << x.d.a;
    const uint32_t nm = x.newmask;
    double m = 0.0;
    if (x.fused) {
        // the round's two steps, one read assignment after another: the
        // assignment's entries (slot a, and slot b of the second step when
        // canonical) are read, the first step's values kept in s_v (indexed
        // by their bits at b and the first step's new slots), and only the
        // second step's entries written
        const uint32_t bbit = 1u << x.d1.a;
        const uint32_t nm1 = x.newmask1;
        const uint32_t X = nm | (x.b_mode == 1 ? bbit : 0u);
        const uint32_t keep = nm & ~bbit;
        const int nta = x.b_mode == 1 ? 2 : 1;
        // every assignment's reads issued before any update
        uint32_t Iv[kTnPairsPerThread];
        T r0v[kTnPairsPerThread][2], r1v[kTnPairsPerThread][2];
#pragma unroll
        for (int k = 0; k < kTnPairsPerThread; ++k) {
            const int64_t p = tblk * kTnThreads + tid + k * stride;
            uint32_t q = static_cast<uint32_t>(p);
            if (x.b_mode == 1) q = tn_pair_index(q, x.b_rank);   // b's place among the canonical bits: 0
            Iv[k] = tn_deposit(q, x);
#pragma unroll
            for (int ta = 0; ta < 2; ++ta) {
                r0v[k][ta] = r1v[k][ta] = TROP ? T(0) : T(1);
                if (p < items && ta < nta && t > 0) {
                    const uint32_t Ib = Iv[k] | (ta ? bbit : 0u);
                    r0v[k][ta] = tab[Ib];
                    r1v[k][ta] = x.a_active ? tab[Ib | abit] : r0v[k][ta];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kTnPairsPerThread; ++k) {
            const int64_t p = tblk * kTnThreads + tid + k * stride;
            if (p >= items) break;
            const uint32_t I = Iv[k];
            const T *r0 = r0v[k], *r1 = r1v[k];
#pragma unroll
            for (int ta = 0; ta < 2; ++ta) {
                if (ta >= nta) break;
                uint32_t c = 0;
                do {
                    const uint32_t idx = I | (ta ? bbit : 0u) | c;
                    const int hh = tn_field(x.d, idx);
                    T v;
                    if (TROP)
                        v = min(r0[ta] + hh, r1[ta] - hh);
                    else
                        v = tn_pair_sum(r0[ta], w[kTnHMax + hh], r1[ta], w[kTnHMax - hh], scale);
                    s_v[tn_extract(idx, X)][tid] = v;
                    c = (c - nm) & nm;
                } while (c != 0);
            }
            uint32_t c0 = 0;
            do {
                const uint32_t B = I | c0;
                const T u0 = s_v[tn_extract(B, X)][tid];
                const T u1 = x.b_mode ? s_v[tn_extract(B | bbit, X)][tid] : u0;
                uint32_t c1 = 0;
                do {
                    const uint32_t O = B | c1;
                    const int hh = tn_field(x.d1, O);
                    T v;
                    if (TROP) {
                        v = min(u0 + hh, u1 - hh);
                    } else {
                        v = tn_pair_sum(u0, w[kTnHMax + hh], u1, w[kTnHMax - hh], 1.0);
                        m = fmax(m, static_cast<double>(v));
                    }
                    tab[O] = v;
                    c1 = (c1 - nm1) & nm1;
                } while (c1 != 0);
                c0 = (c0 - keep) & keep;
            } while (c0 != 0);
        }
    } else {
        // the field splits into the part from canonical slots (once per read) and
        // the part from the new slots (per combination, from s_hn)
        TnDesc db = x.d;
        int n_new = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d)
            if ((nm >> ((db.slots >> (5 * d)) & 31u)) & 1u) db.J[d] = 0;
        for (uint32_t b = nm; b; b &= b - 1) ++n_new;
        if (tid < (1 << n_new)) {
            // combination tid: the bits of tid deposited into the new slots, the
            // tid-th subset in increasing order, as the update loop visits them
            uint32_t c = 0;
            int used = 0;
            for (int b = 0; b < 32; ++b)
                if ((nm >> b) & 1u) c |= ((static_cast<uint32_t>(tid) >> used++) & 1u) << b;
            int hn = 0;
            for (int d = 0; d < 6; ++d) {
                const uint32_t sl = (x.d.slots >> (5 * d)) & 31u;
                if ((nm >> sl) & 1u) hn += x.d.J[d] * (1 - 2 * static_cast<int>((c >> sl) & 1u));
            }
            s_hn[tid] = hn;
        }
        __syncthreads();
        // rounds of kTnReadsInFlight reads (all issued before any update), up to
        // kTnPairsPerThread reads per thread
        for (int r0 = 0; r0 < kTnPairsPerThread; r0 += kTnReadsInFlight) {
            if (tblk * kTnThreads + r0 * stride >= items) break;   // uniform over the work group
            uint32_t I[kTnReadsInFlight];
            T t0[kTnReadsInFlight], t1[kTnReadsInFlight];
#pragma unroll
            for (int r = 0; r < kTnReadsInFlight; ++r) {
                const int64_t p = tblk * kTnThreads + tid + (r0 + r) * stride;
                I[r] = tn_deposit(static_cast<uint32_t>(p), x);
                t0[r] = t1[r] = TROP ? T(0) : T(1);
                if (p < items && t > 0) {
                    t0[r] = tab[I[r]];
                    t1[r] = x.a_active ? tab[I[r] | abit] : t0[r];
                }
            }
#pragma unroll
            for (int r = 0; r < kTnReadsInFlight; ++r) {
                const int64_t p = tblk * kTnThreads + tid + (r0 + r) * stride;
                if (p >= items) break;
                const int hb = tn_field_raw(db, I[r]);
                uint32_t c = 0;
                int kc = 0;
                do {
                    const uint32_t O = I[r] | c;
                    const int hh = min(max(hb + s_hn[kc++], -kTnHMax), kTnHMax);
                    T v;
                    if (TROP) {
                        v = min(t0[r] + hh, t1[r] - hh);
                    } else {
                        v = tn_pair_sum(t0[r], w[kTnHMax + hh], t1[r], w[kTnHMax - hh], scale);
                        m = fmax(m, static_cast<double>(v));
                    }
                    tab[O] = v;
                    c = (c - nm) & nm;
                } while (c != 0);
            }
        }
    }
    if (!TROP) {
        const int e = wave_max_int(m > 0.0 ? ilogb(m) : INT_MIN);
        if ((tid & 63) == 0) s_emax[tid >> 6] = e;
        __syncthreads();
        if (tid == 0) {
            int em = INT_MIN;
            for (int i = 0; i < kTnThreads / 64; ++i) em = max(em, s_emax[i]);
            atomicMax(&bt.emax[tix * bt.steps + t], em);
        }
    }
}

template <bool TROP>
__global__ void k_tn_hbm_final(TnJob jb, TnBatch bt)
{
    using T = typename std::conditional<TROP, int32_t, double>::type;
    const int64_t tix = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int nk = bt.k1 - bt.k0;
    if (tix >= static_cast<int64_t>(bt.nb) * nk * 2) return;
    const int cv = static_cast<int>(tix & 1);
    const int k = bt.k0 + static_cast<int>((tix >> 1) % nk);
    const int bi = static_cast<int>((tix >> 1) / nk);
    const TnTab tb = bt.tabs[tix];
    const T *tab = reinterpret_cast<const T *>(bt.tables) + tb.off;
    double r;
    if (TROP) {
        r = static_cast<double>(static_cast<int64_t>(tab[0]) + bt.es[tix]);
    } else {
        int64_t e_sum = 0;
        for (int t = 0; t + 1 < tb.n_rounds; ++t) e_sum += bt.emax[tix * bt.steps + t];
        r = tn_log_result(static_cast<double>(tab[0]), e_sum, jb.beta, bt.es[tix]);
    }
    jb.res[(static_cast<int64_t>(bt.b0 + bi) * bt.n_items_q + bt.res_k0 + k) * 2 + cv] = r;
}

// ---- decisions ----------------------------------------------------------------

template <bool TROP>
__global__ void k_tn_decide(TnJob jb, int item0, int n_items_q, int n_inst)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n_inst) * n_items_q) return;
    const int inst = static_cast<int>(t / n_items_q);
    const int k = static_cast<int>(t - static_cast<int64_t>(inst) * n_items_q);
    const double zp = jb.res[t * 2], zm = jb.res[t * 2 + 1];
    const double r = TROP ? zm - zp : zp - zm;
    const int64_t g = static_cast<int64_t>(inst) * jb.N + jb.items[item0 + k].site;
    jb.dec[g] = r >= 0.0 ? 1 : -1;
    if (jb.score) jb.score[g] = r;
}

__global__ void k_tn_zero(int8_t *p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---- host side -----------------------------------------------------------------

inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t{255}; }

int64_t res_bytes(const sg_tn_plan &p, int n_inst)
{
    return align256(static_cast<int64_t>(p.max_items) * n_inst * 2 * sizeof(double));
}

// workspace of a batch of nk items: headers, descriptors, work-group
// prefixes, exponents, energies, tables
int64_t batch_bytes(int64_t tables, int64_t entries, int steps, int64_t nk)
{
    return align256(tables * static_cast<int64_t>(sizeof(TnTab))) +
           align256(tables * steps * static_cast<int64_t>(sizeof(TnDescX))) + align256(steps * (nk + 1) * 4) +
           align256(tables * steps * 4) + align256(tables * 4) + align256(entries * 8);
}

int lds_bytes(const TnPhase &P, bool trop, int &tab_bytes)
{
    const int ent = 1 << P.lds_bits;
    tab_bytes = static_cast<int>(align256(static_cast<int64_t>(ent) * (trop ? 4 : 8)));
    return tab_bytes + P.lds_steps * static_cast<int>(sizeof(TnDesc)) + kTnWeights * 8 + 2 * (kTnThreads / 64) * 4;
}

int upload(sg_tn_plan &p)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SG_EDEVICE, "sg_tn_decimate: hipGetDevice");
    std::lock_guard<std::mutex> lock(p.mu);
    if (p.device >= 0) {
        if (p.device != dev)
            return fail(SG_EINVAL, "sg_tn_decimate: the plan was uploaded to device %d, current is %d", p.device, dev);
        return SG_OK;
    }
    auto put = [](void **d, const void *h, size_t n) {
        if (n == 0) n = 8;
        if (hipMalloc(d, n) != hipSuccess) return false;
        return h == nullptr || hipMemcpy(*d, h, n, hipMemcpyHostToDevice) == hipSuccess;
    };
    const bool ok = put(&p.d_shapes, p.shapes.data(), p.shapes.size() * sizeof(TnShape)) &&
                    put(&p.d_steps, p.steps.empty() ? nullptr : p.steps.data(), p.steps.size() * sizeof(TnStep)) &&
                    put(&p.d_rounds, p.rounds.empty() ? nullptr : p.rounds.data(), p.rounds.size() * sizeof(TnRound)) &&
                    put(&p.d_items, p.items.data(), p.items.size() * sizeof(TnItem)) &&
                    put(&p.d_entry_pre, p.hbm_entry_pre.data(), p.hbm_entry_pre.size() * sizeof(int64_t));
    if (!ok) {
        for (void **d : {&p.d_shapes, &p.d_steps, &p.d_rounds, &p.d_items, &p.d_entry_pre})
            if (*d) (void)hipFree(*d), *d = nullptr;
        return fail(SG_ENOMEM, "sg_tn_decimate: uploading the plan");
    }
    // the largest LDS work group of the plan
    int need = 0;
    for (const TnPhase &P : p.phases) {
        int tb;
        if (P.n_lds) need = std::max(need, lds_bytes(P, false, tb));
    }
    if (need > 0) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_tn_lds<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, need) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_tn_lds<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, need) != hipSuccess)
            return fail(SG_EDEVICE, "sg_tn_decimate: LDS attribute (%d bytes)", need);
    }
    hipStream_t side = nullptr, side2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, fork2 = nullptr, join2 = nullptr;
    if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&side2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&fork2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&join2, hipEventDisableTiming) != hipSuccess) {
        for (hipStream_t x : {side, side2})
            if (x) (void)hipStreamDestroy(x);
        for (hipEvent_t x : {fork, join, fork2, join2})
            if (x) (void)hipEventDestroy(x);
        return fail(SG_EDEVICE, "sg_tn_decimate: side streams");
    }
    p.side = side;
    p.fork = fork;
    p.join = join;
    p.side2 = side2;
    p.fork2 = fork2;
    p.join2 = join2;
    p.device = dev;
    return SG_OK;
}

template <bool TROP>
int run(sg_tn_plan &p, const sg_tn_args &a, hipStream_t st)
{
    TnJob jb{};
    jb.J = a.J;
    jb.dec = a.spins_out;
    jb.score = a.score_out;
    jb.shapes = static_cast<const TnShape *>(p.d_shapes);
    jb.steps = static_cast<const TnStep *>(p.d_steps);
    jb.rounds = static_cast<const TnRound *>(p.d_rounds);
    jb.items = static_cast<const TnItem *>(p.d_items);
    jb.res = static_cast<double *>(a.workspace);
    jb.L = p.L;
    jb.h = p.h;
    jb.l = p.l;
    jb.N = static_cast<int64_t>(p.L) * p.L * p.L;
    jb.beta = a.beta;
    // fused rounds keep two steps' growth before a renormalisation: bounded
    // for beta <= SG_TN_FUSE_BETA_MAX (the min-plus form never overflows)
    jb.fuse = (TROP || a.beta <= SG_TN_FUSE_BETA_MAX) ? 1 : 0;
    TnWeights wt{};
    for (int k = -kTnHMax; k <= kTnHMax; ++k) wt.w[k + kTnHMax] = TROP ? 0.0 : std::exp(-a.beta * k);
    const int n_inst = a.n_inst;
    char *heavy = static_cast<char *>(a.workspace) + res_bytes(p, n_inst);
    const int64_t cap = a.workspace_bytes - res_bytes(p, n_inst);

    (void)hipGetLastError();
    const int64_t nz = static_cast<int64_t>(n_inst) * jb.N;
    hipLaunchKernelGGL(k_tn_zero, dim3(static_cast<uint32_t>((nz + 255) / 256)), dim3(256), 0, st, a.spins_out, nz);
    for (const TnPhase &P : p.phases) {
        const int n_items_q = P.n_lds + P.n_hbm;
        if (n_items_q == 0) continue;
        // with both tiers present, the LDS tier runs on the side stream
        // beside the workspace tier and joins before the decisions
        const bool both = P.n_lds && P.n_hbm;
        const hipStream_t lst = both ? static_cast<hipStream_t>(p.side) : st;
        if (both && (hipEventRecord(static_cast<hipEvent_t>(p.fork), st) != hipSuccess ||
                     hipStreamWaitEvent(lst, static_cast<hipEvent_t>(p.fork), 0) != hipSuccess))
            return fail(SG_EDEVICE, "sg_tn_decimate: fork");
        if (P.n_lds) {
            int tb;
            const int bytes = lds_bytes(P, TROP, tb);
            hipLaunchKernelGGL(k_tn_lds<TROP>, dim3(static_cast<uint32_t>(n_inst) * P.n_lds * 2), dim3(kTnThreads),
                               bytes, lst, jb, wt, P.item0, n_items_q, P.n_lds, tb, P.lds_steps);
        }
        if (both && hipEventRecord(static_cast<hipEvent_t>(p.join), lst) != hipSuccess)
            return fail(SG_EDEVICE, "sg_tn_decimate: join");
        if (P.n_hbm) {
            const int64_t *epre = p.hbm_entry_pre.data() + P.hbm0;
            const int steps = P.hbm_steps;
            const int64_t inst_bytes = batch_bytes(2 * P.n_hbm, epre[P.n_hbm], steps, P.n_hbm);
            // batches: whole instances when one fits, else item ranges of one instance
            struct Range { int b0, nb, k0, k1; };
            std::vector<Range> batches;
            // the most work groups a step launch of one instance can need
            int64_t inst_blocks = 0;
            for (int k = 0; k < P.n_hbm; ++k)
                inst_blocks += 2 * tn_table_blocks(p.shapes[p.items[P.item0 + P.n_lds + k].shape].max_base);
            const int max_per = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_inst, INT32_MAX / inst_blocks)));
            if (inst_bytes <= cap) {
                int per = 1;
                while (per < max_per &&
                       batch_bytes(2 * P.n_hbm * int64_t{per + 1}, epre[P.n_hbm] * (per + 1), steps, P.n_hbm) <= cap)
                    ++per;
                for (int b = 0; b < n_inst; b += per)
                    for (int k0 = 0; k0 < P.n_hbm; k0 += kTnThreads)
                        batches.push_back({b, std::min(per, n_inst - b), k0, std::min(P.n_hbm, k0 + kTnThreads)});
            } else {
                for (int b = 0; b < n_inst; ++b)
                    for (int k0 = 0; k0 < P.n_hbm;) {
                        int k1 = k0 + 1;
                        while (k1 < P.n_hbm && k1 - k0 < kTnThreads &&
                               batch_bytes(2 * int64_t{k1 + 1 - k0}, epre[k1 + 1] - epre[k0], steps, k1 + 1 - k0) <= cap)
                            ++k1;
                        batches.push_back({b, 1, k0, k1});
                        k0 = k1;
                    }
            }
            // a batch runs as two halves (of its instances, or of one
            // instance's items), the second on the plan's second stream with
            // its own part of the workspace
            auto range_bytes = [&](const Range &R) {
                return batch_bytes(int64_t{2} * R.nb * (R.k1 - R.k0), (epre[R.k1] - epre[R.k0]) * R.nb, steps,
                                   R.k1 - R.k0);
            };
            struct Unit { Range a, b; bool pair; };
            std::vector<Unit> units;
            for (const Range &R : batches) {
                const Range A{R.b0, R.nb / 2, R.k0, R.k1}, B{R.b0 + R.nb / 2, R.nb - R.nb / 2, R.k0, R.k1};
                if (R.nb >= 2 && range_bytes(A) + range_bytes(B) <= cap) {
                    units.push_back({A, B, true});
                    continue;
                }
                // one instance: its items in two halves of about equal entries
                if (R.nb == 1 && R.k1 - R.k0 >= 2) {
                    int km = R.k0 + 1;
                    while (km + 1 < R.k1 && 2 * (epre[km] - epre[R.k0]) < epre[R.k1] - epre[R.k0]) ++km;
                    const Range A1{R.b0, 1, R.k0, km}, B1{R.b0, 1, km, R.k1};
                    if (range_bytes(A1) + range_bytes(B1) <= cap) {
                        units.push_back({A1, B1, true});
                        continue;
                    }
                }
                units.push_back({R, R, false});
            }
            auto launch_batch = [&](const Range &R, char *base, hipStream_t bs) {
                TnBatch bt{};
                bt.item_hbm0 = P.item0 + P.n_lds;
                bt.res_k0 = P.n_lds;
                bt.n_items_q = n_items_q;
                bt.k0 = R.k0;
                bt.k1 = R.k1;
                bt.b0 = R.b0;
                bt.nb = R.nb;
                bt.steps = steps;
                bt.entry_pre = static_cast<const int64_t *>(p.d_entry_pre) + P.hbm0;
                bt.ents_per_inst = epre[R.k1] - epre[R.k0];
                const int64_t nt = static_cast<int64_t>(R.nb) * (R.k1 - R.k0) * 2;
                char *q = base;
                bt.tabs = reinterpret_cast<TnTab *>(q);
                q += align256(nt * static_cast<int64_t>(sizeof(TnTab)));
                bt.desc = reinterpret_cast<TnDescX *>(q);
                q += align256(nt * steps * static_cast<int64_t>(sizeof(TnDescX)));
                bt.blkpre = reinterpret_cast<int32_t *>(q);
                q += align256(static_cast<int64_t>(steps) * (R.k1 - R.k0 + 1) * 4);
                bt.emax = reinterpret_cast<int32_t *>(q);
                q += align256(nt * steps * 4);
                bt.es = reinterpret_cast<int32_t *>(q);
                q += align256(nt * 4);
                bt.tables = q;
                int max_rounds = 0;
                for (int k = R.k0; k < R.k1; ++k) {
                    const TnShape &sh = p.shapes[p.items[bt.item_hbm0 + k].shape];
                    max_rounds = std::max(max_rounds, jb.fuse ? sh.n_rounds : sh.n_steps);
                }
                hipLaunchKernelGGL(k_tn_hbm_prep, dim3(static_cast<uint32_t>((nt * steps + 255) / 256)), dim3(256), 0, bs,
                                   jb, bt);
                hipLaunchKernelGGL(k_tn_hbm_blocks, dim3(static_cast<uint32_t>((steps + 63) / 64)), dim3(64), 0, bs, jb, bt);
                for (int t = 0; t < max_rounds; ++t) {
                    // work groups of one (instance, value) in this round: as k_tn_hbm_blocks
                    int64_t blocks_t = 0;
                    for (int k = R.k0; k < R.k1; ++k) {
                        const TnShape &sh = p.shapes[p.items[bt.item_hbm0 + k].shape];
                        if (t < (jb.fuse ? sh.n_rounds : sh.n_steps))
                            blocks_t += tn_table_blocks(tn_round(p.rounds.data(), p.steps.data(), sh, t, jb.fuse).read_bits);
                    }
                    if (blocks_t == 0) continue;
                    hipLaunchKernelGGL(k_tn_hbm_step<TROP>, dim3(static_cast<uint32_t>(int64_t{R.nb} * 2 * blocks_t)),
                                       dim3(kTnThreads), 0, bs, bt, wt, t, static_cast<int>(blocks_t));
                }
                hipLaunchKernelGGL(k_tn_hbm_final<TROP>, dim3(static_cast<uint32_t>((nt + 63) / 64)), dim3(64), 0,
                                   bs, jb, bt);
            };
            const hipStream_t st2 = static_cast<hipStream_t>(p.side2);
            for (const Unit &U : units) {
                if (!U.pair) {
                    launch_batch(U.a, heavy, st);
                    continue;
                }
                if (hipEventRecord(static_cast<hipEvent_t>(p.fork2), st) != hipSuccess ||
                    hipStreamWaitEvent(st2, static_cast<hipEvent_t>(p.fork2), 0) != hipSuccess)
                    return fail(SG_EDEVICE, "sg_tn_decimate: fork");
                launch_batch(U.a, heavy, st);
                launch_batch(U.b, heavy + range_bytes(U.a), st2);
                if (hipEventRecord(static_cast<hipEvent_t>(p.join2), st2) != hipSuccess ||
                    hipStreamWaitEvent(st, static_cast<hipEvent_t>(p.join2), 0) != hipSuccess)
                    return fail(SG_EDEVICE, "sg_tn_decimate: join");
            }
        }
        if (both && hipStreamWaitEvent(st, static_cast<hipEvent_t>(p.join), 0) != hipSuccess)
            return fail(SG_EDEVICE, "sg_tn_decimate: join");
        const int64_t nd = static_cast<int64_t>(n_inst) * n_items_q;
        hipLaunchKernelGGL(k_tn_decide<TROP>, dim3(static_cast<uint32_t>((nd + 255) / 256)), dim3(256), 0, st, jb,
                           P.item0, n_items_q, n_inst);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return fail(SG_EDEVICE, "sg_tn_decimate: launch failed: %s", hipGetErrorString(err));
    }
    if (a.energy_out)
        for (int b = 0; b < n_inst; ++b) {
            const int rc = launch_energy(a.J + static_cast<int64_t>(b) * 6 * jb.N, p.L, 1,
                                         a.spins_out + static_cast<int64_t>(b) * jb.N, a.energy_out + b, st);
            if (rc != SG_OK) return rc;
        }
    return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int64_t sg_tn_workspace_bytes(const sg_tn_plan *p, int32_t n_inst, int32_t full)
{
    if (!p || n_inst < 1) return fail(SG_EINVAL, "sg_tn_workspace_bytes: plan NULL or n_inst = %d", n_inst);
    clear_error();
    int64_t heavy = 0;
    for (const TnPhase &P : p->phases) {
        if (!P.n_hbm) continue;
        const int64_t *epre = p->hbm_entry_pre.data() + P.hbm0;
        if (full) {
            heavy = std::max(heavy, batch_bytes(int64_t{2} * P.n_hbm * n_inst, epre[P.n_hbm] * n_inst, P.hbm_steps, P.n_hbm));
        } else {
            for (int k = 0; k < P.n_hbm; ++k)
                heavy = std::max(heavy, batch_bytes(2, epre[k + 1] - epre[k], P.hbm_steps, 1));
        }
    }
    return res_bytes(*p, n_inst) + heavy;
}

int sg_tn_plan_destroy(sg_tn_plan *p)
{
    if (!p) return fail(SG_EINVAL, "sg_tn_plan_destroy: NULL plan");
    clear_error();
    for (void *x : {p->side, p->side2})
        if (x) (void)hipStreamSynchronize(static_cast<hipStream_t>(x));
    for (void *d : {p->d_shapes, p->d_steps, p->d_rounds, p->d_items, p->d_entry_pre})
        if (d) (void)hipFree(d);
    for (void *x : {p->side, p->side2})
        if (x) (void)hipStreamDestroy(static_cast<hipStream_t>(x));
    for (void *x : {p->fork, p->join, p->fork2, p->join2})
        if (x) (void)hipEventDestroy(static_cast<hipEvent_t>(x));
    delete p;
    return SG_OK;
}

int sg_tn_decimate(sg_tn_plan *p, const sg_tn_args *a, void *stream)
{
    if (!p || !a) return fail(SG_EINVAL, "sg_tn_decimate: NULL plan or args");
    if (!a->J || !a->spins_out || !a->workspace) return fail(SG_EINVAL, "sg_tn_decimate: NULL J, spins_out or workspace");
    if (a->n_inst < 1 || a->n_inst > (1 << 16)) return fail(SG_EINVAL, "sg_tn_decimate: n_inst = %d", a->n_inst);
    if (!a->tropical && !(a->beta > 0.0 && a->beta <= 14.0))
        return fail(SG_EINVAL, "sg_tn_decimate: beta = %g outside (0, 14]", a->beta);
    const int64_t need = sg_tn_workspace_bytes(p, a->n_inst, 0);
    if (a->workspace_bytes < need)
        return fail(SG_EINVAL, "sg_tn_decimate: workspace %lld bytes < %lld", static_cast<long long>(a->workspace_bytes),
                    static_cast<long long>(need));
    if (reinterpret_cast<uintptr_t>(a->workspace) % 256 != 0)
        return fail(SG_EINVAL, "sg_tn_decimate: workspace must be 256-byte aligned");
    // one LDS-tier work group per (instance, site, value) of a phase
    if (static_cast<int64_t>(a->n_inst) * p->max_items * 2 > INT32_MAX)
        return fail(SG_ERANGE, "sg_tn_decimate: n_inst = %d exceeds one launch", a->n_inst);
    clear_error();
    int rc = upload(*p);
    if (rc != SG_OK) return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    return a->tropical ? run<true>(*p, *a, st) : run<false>(*p, *a, st);
}

}  // extern "C"
