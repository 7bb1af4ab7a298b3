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
    static constexpr int N = L * L * L;
    static constexpr int JDW_EF = 2 * NC * 6 * 2 * C;  // encoded couplings, E and F
    static constexpr int JDW_E = 2 * NC * 6 * C;       // encoded couplings, E only
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

// byte sum of a dword
__device__ __forceinline__ uint32_t byte_sum(uint32_t v)
{
    return (v & 0xFFu) + ((v >> 8) & 0xFFu) + ((v >> 16) & 0xFFu) + (v >> 24);
}

}  // namespace sg
