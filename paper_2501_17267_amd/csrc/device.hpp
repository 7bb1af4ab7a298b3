// device.hpp -- device-side building blocks shared by the sgmi kernels:
// Philox4x32-10, lattice geometry of the colour-split column layout, and the
// packed-byte local-field arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of two
// 32x32->64 products (counter words 0 and 2) with key injection into words
// 1 and 3; the key advances by the Weyl constants between rounds.  The key
// is uniform across a launch, so its schedule stays in scalar registers.
// ---------------------------------------------------------------------------
struct Rand4 {
    uint32_t w[4];
};

__device__ __forceinline__ Rand4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
        const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
        // three-input xor in one gfx950 bitop3 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Rand4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// The same function with the counter split into words fixed for a whole
// anneal (0, 2, 3 and the key) and word 1 (2s + c, the sweep and colour).
// Following each word through the rounds: round 1's products use words 0
// and 2 only; round 2's product of word 2 and round 3's product of word 0
// are again independent of word 1.  philox_pre computes those three products
// once per call site, philox_hp the word-2 part of round 1 shared by all
// calls of a lane, and per (word 1, lane) philox_q0 is the one product that
// all calls of the lane share; philox_finish then needs one product in
// round 3 and two in each of rounds 4..10 (15 instead of 20).
// philox_finish(philox_pre(c0, c2, c3), philox_q0(philox_hp(c2), c1)) ==
// philox10(c0, c1, c2, c3) for the same key.
struct PhiloxPre {
    uint32_t x3;   // round-1 output word 3 (low product of word 0)
    uint32_t y1;   // round-2 output word 1
    uint32_t hr0;  // round-3 high product of word 0
    uint32_t lr0;  // round-3 low product of word 0 (= round-3 output word 3)
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint32_t philox_hp(uint32_t c2, uint32_t k0)
{
    return static_cast<uint32_t>((static_cast<uint64_t>(c2) * kPhiloxM1) >> 32) ^ k0;
}

__device__ __forceinline__ PhiloxPre philox_pre(uint32_t c0, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = static_cast<uint64_t>(c0) * kPhiloxM0;
    const uint64_t p1 = static_cast<uint64_t>(c2) * kPhiloxM1;
    // round 1 (word 0 of its output needs word 1 and is left to the caller)
    const uint32_t x1 = static_cast<uint32_t>(p1);
    const uint32_t x2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
    const uint32_t x3 = static_cast<uint32_t>(p0);
    // round 2: the product of word 2 and the output words 0 and 1
    const uint64_t q1 = static_cast<uint64_t>(x2) * kPhiloxM1;
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(q1 >> 32), x1, k0 + kPhiloxW0, 0x96);
    // round 3: the product of word 0
    const uint64_t r0 = static_cast<uint64_t>(y0) * kPhiloxM0;
    PhiloxPre p;
    p.x3 = x3;
    p.y1 = static_cast<uint32_t>(q1);
    p.hr0 = static_cast<uint32_t>(r0 >> 32);
    p.lr0 = static_cast<uint32_t>(r0);
    return p;
}

// round-2 product of word 0 for word 1 = c1 (shared by the calls of a lane)
__device__ __forceinline__ uint64_t philox_q0(uint32_t hp, uint32_t c1)
{
    return static_cast<uint64_t>(hp ^ c1) * kPhiloxM0;
}

__device__ __forceinline__ Rand4 philox_finish(const PhiloxPre &p, uint64_t q0, uint32_t k0, uint32_t k1)
{
    // round 2, output words 2 and 3
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(q0 >> 32), p.x3, k1 + kPhiloxW1, 0x96);
    const uint32_t y3 = static_cast<uint32_t>(q0);
    // round 3
    const uint64_t r1 = static_cast<uint64_t>(y2) * kPhiloxM1;
    uint32_t c0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(r1 >> 32), p.y1, k0 + 2u * kPhiloxW0, 0x96);
    uint32_t c1 = static_cast<uint32_t>(r1);
    uint32_t c2 = __builtin_amdgcn_bitop3_b32(p.hr0, y3, k1 + 2u * kPhiloxW1, 0x96);
    uint32_t c3 = p.lr0;
    k0 += 3u * kPhiloxW0;
    k1 += 3u * kPhiloxW1;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t a = static_cast<uint64_t>(c0) * kPhiloxM0;
        const uint64_t b = static_cast<uint64_t>(c2) * kPhiloxM1;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(b >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(a >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(b);
        c3 = static_cast<uint32_t>(a);
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    Rand4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// ---------------------------------------------------------------------------
// Colour-split column layout.  For colour c, the sites with x+y+z = c (mod 2)
// form L^2/2 columns indexed col = k + (L/2) y (k = floor(x/2)); a column
// holds its L sites in z order, four per dword, padded to ceil(L/4) dwords.
// Along a column x alternates between 2k and 2k+1, so every neighbour of a
// colour-c site is in a colour-(1-c) column: (k, y) for +-z (shifted by one
// byte), (k, y+-1) for +-y (same byte), and (k, y) or (k+-1, y) for +-x,
// alternating byte by byte.
// Spins are stored one byte per site: 0x00 for +1, 0xFF for -1.
// ---------------------------------------------------------------------------
template <int L>
struct Geo {
    static_assert(L >= 4 && L % 2 == 0, "L must be even and >= 4");
    static constexpr int H = L / 2;              // columns per row of one colour
    static constexpr int NC = H * L;             // columns per colour
    static constexpr int C = (L + 3) / 4;        // dwords per column
    static constexpr int TAIL = L % 4;           // valid bytes of the last dword, 0 = 4
    static constexpr int SPIN_DW = 2 * NC * C;   // dwords of one replica
    // planes of the split column layout: the first CA dwords of a column
    // (a 64- or 128-bit access) and the other CB
    static constexpr int CA = C >= 4 ? 4 : (C >= 2 ? 2 : 1);
    static constexpr int CB = C - CA;
    static constexpr bool SPLIT_COLUMNS = (C == 3 || C == 5 || C == 6);
    static constexpr int N = L * L * L;
    static constexpr int JDW_EF = 2 * NC * 6 * 2 * C;  // encoded couplings, E and F
    static constexpr int JDW_E = 2 * NC * 6 * C;       // encoded couplings, E only
    static constexpr int JDW_3E = 2 * NC * 3 * C;      // E only, forward directions only
    // The odd-stride LDS arrangement of the couplings (kColMajorOdd, with hn
    // halves per direction): where a column's 6*hn*C dwords sit side by
    // side (jside: not 4-dword columns, nor hn*C = 2 or 4), the stride from
    // one column to the next is padded to an odd count; jdw_odd is its size.
    static constexpr bool jside(int hn) { return C != 4 && hn * C != 2 && hn * C != 4; }
    static constexpr int jstride_odd(int hn) { return 6 * hn * C + ((6 * hn * C) % 2 == 0 ? 1 : 0); }
    static constexpr int jdw_odd(int hn) { return 2 * NC * (jside(hn) ? jstride_odd(hn) : 6 * hn * C); }
};

// The coupling of one direction at four sites of a column dword is encoded
// bytewise as E = J + 8 and F = 8 - J (both in [4, 12]).  With n the
// neighbour-spin dword (0x00/0xFF bytes), bfi(n, F, E) selects 8 + J s_nbr
// per byte; six directions sum to V = 48 + h per byte without carries.
// gfx950 v_bitop3_b32: bit i of the result is imm[(a_i << 2) | (b_i << 1) | c_i];
// 0xE4 is "c ? a : b".  Written as the builtin so that the compiler keeps it
// one instruction instead of splitting it into and/andn feeding an add.
__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(a, b, mask, 0xE4);
}

// Kb = 32 + k per byte, k = -s h (the flip costs dE = 2k): 80 - V where the
// own spin is +1 and V - 16 where it is -1.  Every byte stays in [8, 56],
// below 64, so (Kb >> (8b - 2)) & 0x3FF is exactly 4 x byte b: a table
// address in one bitfield extract.
constexpr uint32_t kKbBias = 32;

__device__ __forceinline__ uint32_t field_to_kb(uint32_t own, uint32_t V)
{
    return bfi(own, V - 0x10101010u, 0x50505050u - V);
}

// byte address (4 x Kb byte b) of the threshold entry of site b
template <int B>
__device__ __forceinline__ uint32_t kb_addr(uint32_t kb)
{
    if (B == 0) return (kb << 2) & 0x3FCu;
    return __builtin_amdgcn_ubfe(kb, 8 * B - 2, 10);
}

// LDS a launch of kern may request dynamically: the compute unit's 160 KB
// less what the kernel holds statically (host code)
inline size_t lds_dynamic_cap(const void *kern)
{
    hipFuncAttributes a{};
    const size_t stat = hipFuncGetAttributes(&a, kern) == hipSuccess ? a.sharedSizeBytes : 0;
    return 160 * 1024 - stat;
}

// byte sum of a dword (an unsigned byte dot product with 1, 1, 1, 1)
__device__ __forceinline__ uint32_t byte_sum(uint32_t v)
{
    return __builtin_amdgcn_udot4(v, 0x01010101u, 0u, false);
}

}  // namespace sg
