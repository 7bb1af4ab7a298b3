// sweep.hpp -- the checkerboard Metropolis sweep shared by the
// simulated-annealing and parallel-tempering kernels.
//
// One work unit = one column of one colour of one replica (L sites along z).
// A lane reads the five neighbouring columns of the other colour, forms the
// packed local fields of its column four sites per dword, draws one
// Philox4x32-10 call per dword (four proposals), and applies the accepted
// flips.  Units of the same colour share no bond, so all lanes of a work
// group update one colour at a time between two barriers.
//
// Column arrays (spins of a replica, encoded couplings) come in two layouts:
//   column-major: dword m of column col of colour c at (c*NC + col)*C + m --
//                 a lane's column is contiguous (wide LDS reads); used in LDS;
//   dword-major:  at (c*C + m)*NC + col -- lanes working on adjacent columns
//                 read adjacent dwords, so HBM loads coalesce; used for
//                 arrays that stay in HBM.
#pragma once

#include "device.hpp"

namespace sg {

enum Layout : int { kColMajor = 0, kDwordMajor = 1, kColMajorOdd = 2, kColSplit = 3, kFwd3 = 4 };

// kColSplit (spins in LDS, columns of C = 3, 5 or 6 dwords): the first CA
// dwords of every column (CA = 2 or 4) in one plane, CA dwords per column,
// and the remaining CB = C - CA dwords in a second plane.  A column read is
// then one 64- or 128-bit access plus one of CB dwords, at lane strides of
// CA and CB dwords, instead of C dwords at an odd stride.  (Only the spins:
// the same split of the couplings measured slower than their arrangement
// below, whose 128-bit reads already spread over the banks.)

// index of dword m of column col, colour c, in a replica's spin array
template <int L, int LAY>
__device__ __forceinline__ int spin_at(int c, int col, int m)
{
    using G = Geo<L>;
    if (LAY == kDwordMajor) return (c * G::C + m) * G::NC + col;
    if (LAY == kColSplit)
        return m < G::CA ? (c * G::NC + col) * G::CA + m
                         : 2 * G::NC * G::CA + (c * G::NC + col) * G::CB + (m - G::CA);
    return (c * G::NC + col) * G::C + m;
}

// index of coupling dword m of column col, colour c, direction d, half h
// (0: E = J + 8, 1: F = 8 - J); HN = 2 when both halves are stored.
// In LDS (kColMajor) a lane reads, per direction, the C dwords of its own
// column, and the lanes of a wave read adjacent columns.  The arrangement
// is chosen per column length so that those reads are single wide accesses
// and the wave's addresses spread over all LDS banks:
//   C = 4:          one plane per (colour, direction, half); columns 16 B
//                   apart (128-bit reads, consecutive lanes consecutive);
//   HN*C = 2 or 4:  one plane per (colour, direction) with E and F of a
//                   column side by side (one 64/128-bit read for both);
//   otherwise:      all twelve (direction, half) blocks of a column side by
//                   side; a column stride of 6*HN*C dwords (36, 60, 72 ...)
//                   already lands successive lanes on distinct banks.
// kColMajorOdd is kColMajor with that last stride padded to an odd count
// (19 instead of 18 at L = 12 with E only).  It serves the PT kernels: their
// sweep is bound by LDS, and at L = 12 the padding made it 2 to 3 % faster;
// the annealing kernel, bound by VALU, ran 8 % slower with it (E and F,
// stride 37), so it keeps kColMajor.
template <int L, int HN>
__device__ __forceinline__ constexpr int lds_jmode()
{
    return Geo<L>::C == 4 ? 0 : ((HN * Geo<L>::C == 2 || HN * Geo<L>::C == 4) ? 1 : 2);
}
static_assert(Geo<12>::jside(1) && Geo<12>::jstride_odd(1) == 19 && !Geo<16>::jside(1) && !Geo<8>::jside(2) &&
                  Geo<10>::jside(2),
              "Geo::jside is mode 2 of lds_jmode");

// kFwd3 (couplings in LDS for lattices whose six directions would not fit):
// E bytes of the three forward directions only (d = 0, 2, 4: +x, +y, +z),
// dword-major; a site's backward coupling is its backward neighbour's
// forward one (Column::field_sum).
template <int L, int HN, int LAY>
__device__ __forceinline__ int coupling_at(int c, int col, int d, int h, int m)
{
    using G = Geo<L>;
    if (LAY == kFwd3) return ((c * 3 + d / 2) * G::C + m) * G::NC + col;
    if (LAY == kDwordMajor) return (((c * 6 + d) * HN + h) * G::C + m) * G::NC + col;
    constexpr int mode = lds_jmode<L, HN>();
    if (mode == 0) return (((c * 6 + d) * HN + h) * G::NC + col) * G::C + m;
    if (mode == 1) return ((c * 6 + d) * G::NC + col) * HN * G::C + h * G::C + m;
    if (LAY == kColMajorOdd) return (c * G::NC + col) * G::jstride_odd(HN) + (d * HN + h) * G::C + m;
    return ((c * G::NC + col) * 6 + d) * HN * G::C + h * G::C + m;
}

template <int L, bool JF, int SLAY = kColMajor, int JLAY = kColMajor>
struct Column {
    using G = Geo<L>;
    static constexpr int C = G::C;
    static constexpr int H = G::H;
    static constexpr int NC = G::NC;
    static constexpr int HN = JF ? 2 : 1;

    // valid-byte mask of dword m (the last dword of a column is half used
    // when L = 2 mod 4)
    __device__ static constexpr uint32_t valid(int m)
    {
        return (G::TAIL != 0 && m == C - 1) ? 0x0000FFFFu : 0xFFFFFFFFu;
    }

    struct Nbr {
        int self, xp, xm, yp, ym;  // neighbouring columns of the other colour
        uint32_t even_x;           // bytes whose x is even
    };

    __device__ static Nbr neighbours(int c, int col)
    {
        const int k = col % H;
        const int y = col / H;
        const int kp = (k + 1 == H) ? 0 : k + 1;
        const int km = (k == 0) ? H - 1 : k - 1;
        const int yp = (y + 1 == L) ? 0 : y + 1;
        const int ym = (y == 0) ? L - 1 : y - 1;
        Nbr n;
        n.self = col;
        n.xp = kp + H * y;
        n.xm = km + H * y;
        n.yp = k + H * yp;
        n.ym = k + H * ym;
        // along a column x alternates between 2k and 2k+1: bytes where x is
        // even take the +x neighbour from column k and the -x one from k-1
        n.even_x = ((y + c) & 1) ? 0xFF00FF00u : 0x00FF00FFu;
        return n;
    }

    // sum over the six directions of 8 + J s_nbr, per byte (n: the column's
    // neighbours, as seen from colour c)
    __device__ static uint32_t field_sum(const uint32_t *jl, int c, int col, int m, const uint32_t (&nb)[6],
                                         const Nbr &n)
    {
        uint32_t V = 0;
        if constexpr (JLAY == kFwd3) {
            static_assert(!JF, "the forward-only arrangement holds E only");
            // backward couplings from the other colour's columns, as the
            // backward neighbour spins are gathered: -x from column k-1 where
            // x is even and from the same index where it is odd, -y from
            // y-1, -z from the site below (one byte down the same column)
            const int oc = c ^ 1;
            uint32_t E[6];
            E[0] = jl[coupling_at<L, 1, kFwd3>(c, col, 0, 0, m)];
            E[2] = jl[coupling_at<L, 1, kFwd3>(c, col, 2, 0, m)];
            E[4] = jl[coupling_at<L, 1, kFwd3>(c, col, 4, 0, m)];
            E[1] = bfi(n.even_x, jl[coupling_at<L, 1, kFwd3>(oc, n.xm, 0, 0, m)],
                       jl[coupling_at<L, 1, kFwd3>(oc, n.self, 0, 0, m)]);
            E[3] = jl[coupling_at<L, 1, kFwd3>(oc, n.ym, 2, 0, m)];
            const uint32_t zc = jl[coupling_at<L, 1, kFwd3>(oc, n.self, 4, 0, m)];
            if (G::TAIL != 0 && m == 0)
                E[5] = __builtin_amdgcn_perm(zc, jl[coupling_at<L, 1, kFwd3>(oc, n.self, 4, 0, C - 1)], 0x06050401u);
            else
                E[5] = __builtin_amdgcn_alignbyte(zc, jl[coupling_at<L, 1, kFwd3>(oc, n.self, 4, 0, m > 0 ? m - 1 : C - 1)],
                                                  3);
#pragma unroll
            for (int d = 0; d < 6; ++d) V += bfi(nb[d], 0x10101010u - E[d], E[d]);
            return V;
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const uint32_t E = jl[coupling_at<L, HN, JLAY>(c, col, d, 0, m)];
            const uint32_t F = JF ? jl[coupling_at<L, HN, JLAY>(c, col, d, 1, m)] : 0x10101010u - E;
            V += bfi(nb[d], F, E);
        }
        return V;
    }

    // Kb (= 32 + k per byte) of every dword of column `col` of colour c.
    // rep: spins of the replica; jl: couplings.  own receives the column.
    __device__ static void fields(const uint32_t *rep, const uint32_t *jl, int c, int col, uint32_t (&own)[C],
                                  uint32_t (&kb)[C])
    {
        fields_n(rep, jl, c, col, neighbours(c, col), own, kb);
    }

    __device__ static void fields_n(const uint32_t *rep, const uint32_t *jl, int c, int col, const Nbr &n,
                                    uint32_t (&own)[C], uint32_t (&kb)[C])
    {
        const int oc = c ^ 1;
        uint32_t sv[C], xp[C], xm[C], yv[C], ymv[C];
#pragma unroll
        for (int m = 0; m < C; ++m) {
            sv[m] = rep[spin_at<L, SLAY>(oc, n.self, m)];
            xp[m] = rep[spin_at<L, SLAY>(oc, n.xp, m)];
            xm[m] = rep[spin_at<L, SLAY>(oc, n.xm, m)];
            yv[m] = rep[spin_at<L, SLAY>(oc, n.yp, m)];
            ymv[m] = rep[spin_at<L, SLAY>(oc, n.ym, m)];
            own[m] = rep[spin_at<L, SLAY>(c, col, m)];
        }
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
            const uint32_t nb[6] = {bfi(n.even_x, sv[m], xp[m]), bfi(n.even_x, xm[m], sv[m]), yv[m], ymv[m], zp, zm};
            kb[m] = field_to_kb(own[m], field_sum(jl, c, col, m, nb, n));
        }
    }

    // The six neighbour bytes (+x, -x, +y, -y, +z, -z) of the four sites of
    // dword m of colour-c column col, gathered from the colour-(1-c)
    // columns of a byte array in the column layout (spins, or any per-site
    // byte mask laid out the same way)
    __device__ static void nbr_dwords_n(const uint32_t *rep, int c, const Nbr &n, int m, uint32_t (&nb)[6])
    {
        const int oc = c ^ 1;
        const uint32_t s_m = rep[spin_at<L, SLAY>(oc, n.self, m)];
        uint32_t zp, zm;
        if (G::TAIL != 0 && m == C - 1)
            zp = __builtin_amdgcn_perm(rep[spin_at<L, SLAY>(oc, n.self, 0)], s_m, 0x00000401u);
        else
            zp = __builtin_amdgcn_alignbyte(rep[spin_at<L, SLAY>(oc, n.self, m + 1 < C ? m + 1 : 0)], s_m, 1);
        if (G::TAIL != 0 && m == 0)
            zm = __builtin_amdgcn_perm(s_m, rep[spin_at<L, SLAY>(oc, n.self, C - 1)], 0x06050401u);
        else
            zm = __builtin_amdgcn_alignbyte(s_m, rep[spin_at<L, SLAY>(oc, n.self, m > 0 ? m - 1 : C - 1)], 3);
        nb[0] = bfi(n.even_x, s_m, rep[spin_at<L, SLAY>(oc, n.xp, m)]);
        nb[1] = bfi(n.even_x, rep[spin_at<L, SLAY>(oc, n.xm, m)], s_m);
        nb[2] = rep[spin_at<L, SLAY>(oc, n.yp, m)];
        nb[3] = rep[spin_at<L, SLAY>(oc, n.ym, m)];
        nb[4] = zp;
        nb[5] = zm;
    }

    // Kb of dword m only, loading just what it needs (the streaming path for
    // long columns, where six whole neighbour columns would not fit in
    // registers)
    __device__ static uint32_t field_dword(const uint32_t *rep, const uint32_t *jl, int c, int col, int m,
                                           uint32_t own_m)
    {
        uint32_t nb[6];
        const Nbr n = neighbours(c, col);
        nbr_dwords_n(rep, c, n, m, nb);
        return field_to_kb(own_m, field_sum(jl, c, col, m, nb, n));
    }

    // 0xFF in every byte of dword m of colour-c column col whose coupling in
    // direction d is nonzero (E = J + 8 differs from 8)
    __device__ static uint32_t nonzero_coupling(const uint32_t *jl, int c, int col, int d, int m)
    {
        const uint32_t x = jl[coupling_at<L, HN, JLAY>(c, col, d, 0, m)] ^ 0x08080808u;  // J & 15 per byte
        const uint32_t t = ((x & 0x0F0F0F0Fu) + 0x0F0F0F0Fu) & 0x10101010u;             // bit 4: J != 0
        return (t >> 4) * 0xFFu;
    }

    // columns longer than this are processed dword by dword
    static constexpr bool kStream = C > 6;

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

    // sum of s_i h_i over the valid sites of colour-0 column `col`; summed
    // over all colour-0 columns this is the energy of Eq. 1 (every bond
    // joins a colour-0 and a colour-1 site)
    __device__ static int32_t column_energy_of(const uint32_t *rep, const uint32_t *jl, int col)
    {
        int32_t e = 0;
        if constexpr (kStream) {
            for (int m = 0; m < C; ++m) {
                const uint32_t kbm = field_dword(rep, jl, 0, col, m, rep[spin_at<L, SLAY>(0, col, m)]);
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

    // one dword's four proposals: returns the flip mask, adds to dE.
    // tb: LDS threshold table indexed by Kb = 32 + k (entries 33..32+K hold
    // the thresholds of k = 1..K, later ones are zero); k <= 0 always flips.
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
            // downhill (k <= 0, i.e. 4 Kb <= 128) always; uphill iff u < thr[k]
            const bool acc = (addr[b] <= 4u * kKbBias) | (u.w[b] < t);
            flip |= acc ? (0xFFu << (8 * b)) : 0u;
        }
        if (TRACK) {
            // an accepted flip changes the energy by 2 (Kb - 32).  Read as
            // int8, an accepted byte of `flip` is -1 and a Kb byte (below
            // 64) is itself, so two byte dot products give minus the sum of
            // Kb - 32 over the accepted sites (0xE0 is -32)
            int32_t nh = __builtin_amdgcn_sdot4(static_cast<int32_t>(flip), static_cast<int32_t>(kbm), 0, false);
            nh = __builtin_amdgcn_sdot4(static_cast<int32_t>(flip), static_cast<int32_t>(0xE0E0E0E0u), nh, false);
            dE -= 2 * nh;
        }
        return flip;
    }

    // One Metropolis pass over the column: proposals at every valid site,
    // random words from Philox call (col*C + m, c1, rep_word, chain).
    // Returns the energy change of the column when TRACK, else 0.
    template <bool TRACK>
    __device__ static int32_t metropolis(uint32_t *rep, const uint32_t *jl, const uint32_t *thr, int c, int col,
                                         uint32_t c1, uint32_t rep_word, uint32_t chain, uint32_t k0, uint32_t k1)
    {
        int32_t dE = 0;
        const char *tb = reinterpret_cast<const char *>(thr);
        if constexpr (kStream) {
            // long columns: dword by dword (this colour's updates never feed
            // this colour's fields, so the order does not matter)
            for (int m = 0; m < C; ++m) {
                const int at = spin_at<L, SLAY>(c, col, m);
                const uint32_t own_m = rep[at];
                const uint32_t kbm = field_dword(rep, jl, c, col, m, own_m);
                const Rand4 u = philox10(static_cast<uint32_t>(col * C + m), c1, rep_word, chain, k0, k1);
                rep[at] = own_m ^ accept_dword<TRACK>(kbm, u, tb, m, dE);
            }
            return dE;
        }
        uint32_t own[C], kb[C];
        fields(rep, jl, c, col, own, kb);
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const Rand4 u = philox10(static_cast<uint32_t>(col * C + m), c1, rep_word, chain, k0, k1);
            own[m] ^= accept_dword<TRACK>(kb[m], u, tb, m, dE);
        }
#pragma unroll
        for (int m = 0; m < C; ++m) rep[spin_at<L, SLAY>(c, col, m)] = own[m];
        return dE;
    }

    // A unit whose column and replica stay fixed for a whole anneal: its
    // neighbour columns and the word-1-independent part of the Philox calls
    // of its C dwords (counter (col*C + m, ., rep_word, chain)) are computed
    // once.  Only for columns held whole in registers (not kStream).
    struct Unit {
        Nbr n;            // as seen from colour 0; colour 1 flips even_x
        uint32_t hp;      // philox_hp(rep_word, k0)
        PhiloxPre pre[C];
    };

    __device__ static Unit make_unit(int col, uint32_t rep_word, uint32_t chain, uint32_t k0, uint32_t k1)
    {
        Unit u;
        u.n = neighbours(0, col);
        u.hp = philox_hp(rep_word, k0);
#pragma unroll
        for (int m = 0; m < C; ++m) u.pre[m] = philox_pre(static_cast<uint32_t>(col * C + m), rep_word, chain, k0, k1);
        return u;
    }

    // metropolis() for a prepared unit; c1 = 2s + c.  Same result.
    template <bool TRACK>
    __device__ static int32_t metropolis_unit(uint32_t *rep, const uint32_t *jl, const uint32_t *thr, int c,
                                              const Unit &un, uint32_t c1, uint32_t k0, uint32_t k1)
    {
        static_assert(!kStream, "prepared units hold whole columns");
        int32_t dE = 0;
        const char *tb = reinterpret_cast<const char *>(thr);
        Nbr n = un.n;
        if (c) n.even_x = ~n.even_x;
        uint32_t own[C], kb[C];
        fields_n(rep, jl, c, n.self, n, own, kb);
        const uint64_t q0 = philox_q0(un.hp, c1);
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const Rand4 u = philox_finish(un.pre[m], q0, k0, k1);
            own[m] ^= accept_dword<TRACK>(kb[m], u, tb, m, dE);
        }
#pragma unroll
        for (int m = 0; m < C; ++m) rep[spin_at<L, SLAY>(c, n.self, m)] = own[m];
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

// byte offset of natural site i inside one replica's column array
template <int L, int LAY = kColMajor>
__device__ __forceinline__ int site_byte(int i)
{
    using G = Geo<L>;
    const int x = i % L;
    const int y = (i / L) % L;
    const int z = i / (L * L);
    const int c = (x + y + z) & 1;
    const int col = (x >> 1) + G::H * y;
    return 4 * spin_at<L, LAY>(c, col, z >> 2) + (z & 3);
}

// E and F bytes of dword m of column col, colour c, direction d from the
// natural-order couplings J[6][N] (padding sites: J = 0)
template <int L>
__device__ __forceinline__ void encode_dword(const int8_t *J, int c, int col, int d, int m, uint32_t &e, uint32_t &f)
{
    using G = Geo<L>;
    const int k = col % G::H;
    const int y = col / G::H;
    e = 0;
    f = 0;
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
}

// Fill the LDS couplings (column-major) from natural-order J[6][N] or from
// the encoded HBM buffer (dword-major, E and F) when given.
template <int L, bool JF, int JLAY = kColMajor>
__device__ void load_couplings(uint32_t *jl, const int8_t *J, const uint32_t *jenc, int tid, int nt)
{
    using G = Geo<L>;
    constexpr int C = G::C;
    constexpr int HN = JF ? 2 : 1;
    constexpr int ND = JLAY == kFwd3 ? 3 : 6;   // directions held (forward only: d = 0, 2, 4)
    for (int w = tid; w < 2 * G::NC * ND * C; w += nt) {
        const int m = w % C;
        int t = w / C;
        const int d = JLAY == kFwd3 ? 2 * (t % 3) : t % 6;
        t /= ND;
        const int col = t % G::NC;
        const int c = t / G::NC;
        uint32_t e, f;
        if (jenc) {
            e = jenc[coupling_at<L, 2, kDwordMajor>(c, col, d, 0, m)];
            f = jenc[coupling_at<L, 2, kDwordMajor>(c, col, d, 1, m)];
        } else {
            encode_dword<L>(J, c, col, d, m, e, f);
        }
        jl[coupling_at<L, HN, JLAY>(c, col, d, 0, m)] = e;
        if (JF) jl[coupling_at<L, HN, JLAY>(c, col, d, 1, m)] = f;
    }
}

// Initial spins of one replica: from the init stream or from natural-order
// int8 spins.  The replica's array must be zeroed beforehand (padding).
template <int L, int LAY = kColMajor>
__device__ void load_spins_one(uint8_t *repb, int q, bool init_random, const int8_t *src, uint32_t rep_word,
                               uint32_t chain, uint32_t k0, uint32_t k1)
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
    for (int b = 0; b < 4; ++b) repb[site_byte<L, LAY>(4 * q + b)] = static_cast<uint8_t>(w4[b]);
}

template <int L, int LAY = kColMajor>
__device__ __forceinline__ void store_spins_one(const uint8_t *repb, int q, int8_t *dst)
{
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t s = repb[site_byte<L, LAY>(4 * q + b)] ? 0xFFu : 0x01u;
        v |= s << (8 * b);
    }
    reinterpret_cast<uint32_t *>(dst)[q] = v;
}

}  // namespace sg
