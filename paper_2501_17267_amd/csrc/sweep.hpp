// sweep.hpp -- the LDS-resident checkerboard Metropolis sweep shared by the
// simulated-annealing and parallel-tempering kernels.
//
// One work unit = one column of one colour of one replica (L sites along z).
// A lane loads the five neighbouring columns of the other colour, forms the
// packed local fields of its column four sites per dword, draws one
// Philox4x32-10 call per dword (four proposals), and applies the accepted
// flips.  Units of the same colour share no bond, so all lanes of a work
// group update one colour at a time between two barriers.
#pragma once

#include "device.hpp"

namespace sg {

template <int L, bool JF>
struct Column {
    using G = Geo<L>;
    static constexpr int C = G::C;
    static constexpr int H = G::H;
    static constexpr int NC = G::NC;
    static constexpr int JSTRIDE = JF ? 12 * C : 6 * C;  // dwords of couplings per column

    // valid-byte mask of dword m (the last dword of a column is half used
    // when L = 2 mod 4)
    __device__ static constexpr uint32_t valid(int m)
    {
        return (G::TAIL != 0 && m == C - 1) ? 0x0000FFFFu : 0xFFFFFFFFu;
    }

    // Kb (= 48 + k per byte) of every dword of column `col` of colour c.
    // rep: LDS spins of the replica; jl: LDS couplings.  own receives the
    // column's spin dwords.
    __device__ static void fields(const uint32_t *rep, const uint32_t *jl, int c, int col,
                                  uint32_t (&own)[C], uint32_t (&kb)[C])
    {
        const int k = col % H;
        const int y = col / H;
        const int kp = (k + 1 == H) ? 0 : k + 1;
        const int km = (k == 0) ? H - 1 : k - 1;
        const int yp = (y + 1 == L) ? 0 : y + 1;
        const int ym = (y == 0) ? L - 1 : y - 1;
        const uint32_t *other = rep + (c ^ 1) * NC * C;
        const uint32_t *pS = other + col * C;
        const uint32_t *pXp = other + (kp + H * y) * C;
        const uint32_t *pXm = other + (km + H * y) * C;
        const uint32_t *pYp = other + (k + H * yp) * C;
        const uint32_t *pYm = other + (k + H * ym) * C;
        const uint32_t *pO = rep + c * NC * C + col * C;
        // bytes where x is even (p = 0) take the +x neighbour from column k
        // and the -x neighbour from column k-1
        const uint32_t even_x = ((y + c) & 1) ? 0xFF00FF00u : 0x00FF00FFu;
        uint32_t sv[C], xp[C], xm[C], yv[C], ymv[C];
#pragma unroll
        for (int m = 0; m < C; ++m) {
            sv[m] = pS[m];
            xp[m] = pXp[m];
            xm[m] = pXm[m];
            yv[m] = pYp[m];
            ymv[m] = pYm[m];
            own[m] = pO[m];
        }
        const uint32_t *jc = jl + (c * NC + col) * JSTRIDE;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            uint32_t zp, zm;
            if (G::TAIL != 0 && m == C - 1)
                zp = __builtin_amdgcn_perm(sv[0], sv[C - 1], 0x00000401u);
            else
                zp = __builtin_amdgcn_alignbyte(sv[(m + 1) % C], sv[m], 1);
            if (G::TAIL != 0 && m == 0)
                zm = __builtin_amdgcn_perm(sv[0], sv[C - 1], 0x06050401u);
            else
                zm = __builtin_amdgcn_alignbyte(sv[m], sv[(m + C - 1) % C], 3);
            const uint32_t nxp = bfi(even_x, sv[m], xp[m]);
            const uint32_t nxm = bfi(even_x, xm[m], sv[m]);
            const uint32_t nb[6] = {nxp, nxm, yv[m], ymv[m], zp, zm};
            uint32_t V = 0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                uint32_t E, F;
                if (JF) {
                    E = jc[d * 2 * C + m];
                    F = jc[d * 2 * C + C + m];
                } else {
                    E = jc[d * C + m];
                    F = 0x10101010u - E;
                }
                V += bfi(nb[d], F, E);
            }
            kb[m] = field_to_kb(own[m], V);
        }
    }

    // Kb of dword m of column `col` of colour c, loading only what it needs
    // (the streaming path for long columns, where holding the whole column
    // of six neighbour arrays would exceed the register budget).
    __device__ static uint32_t field_dword(const uint32_t *rep, const uint32_t *jl, int c, int col, int m,
                                           uint32_t own_m)
    {
        const int k = col % H;
        const int y = col / H;
        const int kp = (k + 1 == H) ? 0 : k + 1;
        const int km = (k == 0) ? H - 1 : k - 1;
        const int yp = (y + 1 == L) ? 0 : y + 1;
        const int ym = (y == 0) ? L - 1 : y - 1;
        const uint32_t *other = rep + (c ^ 1) * NC * C;
        const uint32_t *pS = other + col * C;
        const uint32_t even_x = ((y + c) & 1) ? 0xFF00FF00u : 0x00FF00FFu;
        const uint32_t s_m = pS[m];
        uint32_t zp, zm;
        if (G::TAIL != 0 && m == C - 1)
            zp = __builtin_amdgcn_perm(pS[0], s_m, 0x00000401u);
        else
            zp = __builtin_amdgcn_alignbyte(pS[m + 1 < C ? m + 1 : 0], s_m, 1);
        if (G::TAIL != 0 && m == 0)
            zm = __builtin_amdgcn_perm(s_m, pS[C - 1], 0x06050401u);
        else
            zm = __builtin_amdgcn_alignbyte(s_m, pS[m > 0 ? m - 1 : C - 1], 3);
        const uint32_t nb[6] = {bfi(even_x, s_m, other[(kp + H * y) * C + m]),
                                bfi(even_x, other[(km + H * y) * C + m], s_m), other[(k + H * yp) * C + m],
                                other[(k + H * ym) * C + m], zp, zm};
        const uint32_t *jc = jl + (c * NC + col) * JSTRIDE;
        uint32_t V = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            uint32_t E, F;
            if (JF) {
                E = jc[d * 2 * C + m];
                F = jc[d * 2 * C + C + m];
            } else {
                E = jc[d * C + m];
                F = 0x10101010u - E;
            }
            V += bfi(nb[d], F, E);
        }
        return field_to_kb(own_m, V);
    }

    // columns longer than this are processed dword by dword
    static constexpr bool kStream = C > 6;

    // sum of s_i h_i over the valid sites of colour-0 column `col`; summed
    // over all colour-0 columns this is the energy of Eq. 1 (every bond
    // joins a colour-0 and a colour-1 site)
    __device__ static int32_t column_energy_of(const uint32_t *rep, const uint32_t *jl, int col)
    {
        int32_t e = 0;
        if constexpr (kStream) {
            const uint32_t *pO = rep + col * C;
            for (int m = 0; m < C; ++m) {
                const uint32_t kbm = field_dword(rep, jl, 0, col, m, pO[m]);
                const int nvalid = (G::TAIL != 0 && m == C - 1) ? G::TAIL : 4;
                e += static_cast<int32_t>(kKbBias) * nvalid - static_cast<int32_t>(byte_sum(kbm & valid(m)));
            }
        } else {
            uint32_t own[C], kb[C];
            fields(rep, jl, 0, col, own, kb);
            e = column_energy(kb);
        }
        return e;
    }

    // sum over the valid sites of the column of s_i h_i = 32 - Kb
    __device__ static int32_t column_energy(const uint32_t (&kb)[C])
    {
        int32_t e = 0;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int nvalid = (G::TAIL != 0 && m == C - 1) ? G::TAIL : 4;
            e += static_cast<int32_t>(kKbBias) * nvalid - static_cast<int32_t>(byte_sum(kb[m] & valid(m)));
        }
        return e;
    }

    // One Metropolis pass over the column: proposals at every valid site,
    // random words from Philox call (col*C + m, c1, rep_word, chain).
    // thr: LDS table of 32-bit thresholds indexed by Kb = 32 + k.  Entries
    // 33..32+K hold the thresholds of k = 1..K, entries up to 63 beyond K
    // are zero (never accept); k <= 0 always flips without reading the
    // table.  Returns the energy change of the column when TRACK, else 0.
    // one dword's four proposals: returns the flip mask, adds to dE
    template <bool TRACK>
    __device__ static uint32_t accept_dword(uint32_t kbm, const Rand4 &u, const char *tb, int m, int32_t &dE)
    {
        uint32_t addr[4];
        addr[0] = kb_addr<0>(kbm);
        addr[1] = kb_addr<1>(kbm);
        addr[2] = kb_addr<2>(kbm);
        addr[3] = kb_addr<3>(kbm);
        uint32_t flip = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (G::TAIL != 0 && m == C - 1 && b >= G::TAIL) continue;
            const uint32_t t = *reinterpret_cast<const uint32_t *>(tb + addr[b]);
            const bool acc = (addr[b] <= 4u * kKbBias) | (u.w[b] < t);
            flip |= acc ? (0xFFu << (8 * b)) : 0u;
            if (TRACK) dE += acc ? 2 * (static_cast<int32_t>(addr[b] >> 2) - static_cast<int32_t>(kKbBias)) : 0;
        }
        return flip;
    }

    template <bool TRACK>
    __device__ static int32_t metropolis(uint32_t *rep, const uint32_t *jl, const uint32_t *thr, int c,
                                         int col, uint32_t c1, uint32_t rep_word, uint32_t chain,
                                         uint32_t k0, uint32_t k1)
    {
        if constexpr (kStream) {
            // long columns: dword by dword (same proposals, same order of
            // effects: this colour's updates never feed this colour's fields)
            int32_t dE = 0;
            const char *tb = reinterpret_cast<const char *>(thr);
            uint32_t *pO = rep + c * NC * C + col * C;
            for (int m = 0; m < C; ++m) {
                const uint32_t own_m = pO[m];
                const uint32_t kbm = field_dword(rep, jl, c, col, m, own_m);
                const Rand4 u = philox10(static_cast<uint32_t>(col * C + m), c1, rep_word, chain, k0, k1);
                pO[m] = own_m ^ accept_dword<TRACK>(kbm, u, tb, m, dE);
            }
            return dE;
        }
        uint32_t own[C], kb[C];
        fields(rep, jl, c, col, own, kb);
        int32_t dE = 0;
        const char *tb = reinterpret_cast<const char *>(thr);
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const Rand4 u = philox10(static_cast<uint32_t>(col * C + m), c1, rep_word, chain, k0, k1);
            uint32_t addr[4];
            addr[0] = kb_addr<0>(kb[m]);
            addr[1] = kb_addr<1>(kb[m]);
            addr[2] = kb_addr<2>(kb[m]);
            addr[3] = kb_addr<3>(kb[m]);
            uint32_t flip = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (G::TAIL != 0 && m == C - 1 && b >= G::TAIL) continue;
                const uint32_t t = *reinterpret_cast<const uint32_t *>(tb + addr[b]);
                // downhill (k <= 0, i.e. 4 Kb <= 128) always; uphill iff u < thr[k]
                const bool acc = (addr[b] <= 4u * kKbBias) | (u.w[b] < t);
                flip |= acc ? (0xFFu << (8 * b)) : 0u;
                if (TRACK) dE += acc ? 2 * (static_cast<int32_t>(addr[b] >> 2) - static_cast<int32_t>(kKbBias)) : 0;
            }
            own[m] ^= flip;
        }
        uint32_t *pO = rep + c * NC * C + col * C;
#pragma unroll
        for (int m = 0; m < C; ++m) pO[m] = own[m];
        return dE;
    }
};

// ---------------------------------------------------------------------------
// Work-group set-up helpers (natural site order <-> column layout).
// ---------------------------------------------------------------------------

// entries of an LDS threshold table indexed by Kb = 32 + k
constexpr int kThrEntries = 64;

// entry e of the table built from one row thr[0..K-1] (k = e - 32)
__device__ __forceinline__ uint32_t thr_entry(const uint32_t *row, int K, int e)
{
    const int k = e - static_cast<int>(kKbBias);
    if (k <= 0) return 0xFFFFFFFFu;
    return (k <= K) ? row[k - 1] : 0u;
}

// byte offset of natural site i inside one replica's column layout
template <int L>
__device__ __forceinline__ int site_byte(int i)
{
    using G = Geo<L>;
    const int x = i % L;
    const int y = (i / L) % L;
    const int z = i / (L * L);
    const int c = (x + y + z) & 1;
    const int col = (x >> 1) + G::H * y;
    return ((c * G::NC + col) * G::C) * 4 + z;
}

// Fill LDS couplings from natural-order J[6][N] (device) or from the
// pre-encoded buffer (E and F layout) when given.
template <int L, bool JF>
__device__ void load_couplings(uint32_t *jl, const int8_t *J, const uint32_t *jenc, int tid, int nt)
{
    using G = Geo<L>;
    constexpr int C = G::C;
    if (jenc) {
        if (JF) {
            for (int w = tid; w < G::JDW_EF; w += nt) jl[w] = jenc[w];
        } else {
            // keep the E halves only
            for (int w = tid; w < G::JDW_E; w += nt) {
                const int m = w % C;
                const int cd = w / C;  // (c*NC + col)*6 + d
                jl[w] = jenc[cd * 2 * C + m];
            }
        }
        return;
    }
    for (int w = tid; w < 2 * G::NC * 6 * C; w += nt) {
        const int m = w % C;
        int t = w / C;
        const int d = t % 6;
        t /= 6;
        const int col = t % G::NC;
        const int c = t / G::NC;
        const int k = col % G::H;
        const int y = col / G::H;
        uint32_t e = 0, f = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int z = 4 * m + b;
            int jv = 0;
            if (z < L) {
                const int x = 2 * k + ((y + z + c) & 1);
                jv = J[d * G::N + x + L * (y + L * z)];
            }
            e |= static_cast<uint32_t>(8 + jv) << (8 * b);
            f |= static_cast<uint32_t>(8 - jv) << (8 * b);
        }
        const int base = ((c * G::NC + col) * 6 + d);
        if (JF) {
            jl[base * 2 * C + m] = e;
            jl[base * 2 * C + C + m] = f;
        } else {
            jl[base * C + m] = e;
        }
    }
}

// Initial spins of one replica: from the init stream or from natural-order
// int8 spins.  The replica's LDS block must be zeroed beforehand (padding).
template <int L>
__device__ void load_spins_one(uint8_t *repb, int q, bool init_random, const int8_t *src,
                               uint32_t rep_word, uint32_t chain, uint32_t k0, uint32_t k1)
{
    uint32_t w4[4];
    if (init_random) {
        const Rand4 u = philox10(static_cast<uint32_t>(q), 0xFFFFFFFFu, rep_word, chain, k0, k1);
#pragma unroll
        for (int b = 0; b < 4; ++b) w4[b] = (u.w[b] >> 31) ? 0xFFu : 0u;
    } else {
        const uint32_t v = reinterpret_cast<const uint32_t *>(src)[q];
#pragma unroll
        for (int b = 0; b < 4; ++b) w4[b] = (((v >> (8 * b)) & 0x80u) != 0) ? 0xFFu : 0u;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) repb[site_byte<L>(4 * q + b)] = static_cast<uint8_t>(w4[b]);
}

template <int L>
__device__ __forceinline__ void store_spins_one(const uint8_t *repb, int q, int8_t *dst)
{
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t s = repb[site_byte<L>(4 * q + b)] ? 0xFFu : 0x01u;
        v |= s << (8 * b);
    }
    reinterpret_cast<uint32_t *>(dst)[q] = v;
}

}  // namespace sg
