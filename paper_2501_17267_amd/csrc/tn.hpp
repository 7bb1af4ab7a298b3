// tn.hpp -- plan of the tensor-network fragment decimation, shared by the
// host planner (tn_plan.cpp) and the kernels (tn.hip).
//
// A fragment's free spins (all but the centre, which each table fixes at
// one value) are eliminated one by one.  The running table is indexed by
// the "active" spins: free spins not yet eliminated that share a bond with
// an eliminated one (or are about to be eliminated).  Every active spin owns
// one bit ("slot") of the table index; bit value 0 means s = +1, 1 means
// s = -1.  A slot that no spin owns is a dimension along which the table is
// constant, so a spin can take a free slot at any time without touching the
// table.  Eliminating spin v (slot a) replaces, for every index I with bit
// a = 0, both T[I] and T[I | 1<<a] by
//   T[I] w(+1) + T[I | 1<<a] w(-1),   w(s) = exp(-beta s h_v),
// where h_v sums J_vu s_u over v's bonds to active, fixed and centre spins
// (bonds to spins eliminated earlier were counted then).  The tropical form
// uses min(T[I] + h_v, T[I | 1<<a] - h_v).  After the last step the table
// is constant: Z (or the least energy) of the free spins given the centre.
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include "sgmi.h"

namespace sg {

constexpr int8_t kTnConst = -1;    // fixed (decimated earlier) neighbour
constexpr int8_t kTnCentre = -2;   // the centre
constexpr int8_t kTnNone = -3;     // outside the fragment or already eliminated

struct TnStep {
    int16_t lv;        // local index of the eliminated spin, lx + l (ly + l lz)
    uint8_t a;         // its slot
    uint8_t pad;
    int8_t code[6];    // per direction +x,-x,+y,-y,+z,-z: slot (>= 0) or kTn*
    int16_t pad2;
};
static_assert(sizeof(TnStep) == 12, "TnStep layout");

struct TnShape {
    int32_t W;         // table bits (2^W entries)
    int32_t n_steps;   // eliminations
    int32_t step0;     // first step in the step array
    int8_t ccode[6];   // the centre's neighbours: kTnConst (fixed) or kTnNone
    int16_t pad;
};
static_assert(sizeof(TnShape) == 20, "TnShape layout");

struct TnItem {
    int32_t site;      // global index of the centre
    int32_t shape;
};

struct TnPhase {
    int32_t item0;     // items of the phase: [item0, item0 + n_lds) in LDS,
    int32_t n_lds;     //   then n_hbm in the workspace
    int32_t n_hbm;
    int32_t lds_bits;  // largest LDS table of the phase
    int32_t lds_steps; // most steps of an LDS item
    int32_t hbm_steps; // most steps of a workspace item
    int64_t hbm0;      // first entry of the phase in the workspace prefix arrays
};

}  // namespace sg

struct sg_tn_plan {
    int32_t L = 0, h = 0, l = 0, order = 0, lds_bits = 0;
    std::vector<sg::TnShape> shapes;
    std::vector<sg::TnStep> steps;
    std::vector<sg::TnItem> items;
    std::vector<sg::TnPhase> phases;
    // workspace items in phase order: table-entry and block prefixes of one
    // instance (both centre values), per phase relative to the phase start
    std::vector<int64_t> hbm_entry_pre;   // [n_hbm_total + n_phases]
    std::vector<int64_t> hbm_block_pre;
    int32_t max_bits = 0, max_steps = 0, n_lds = 0, n_hbm = 0, max_items = 0;
    double pair_updates = 0;
    // device copies (first decimation)
    std::mutex mu;
    int device = -1;
    void *d_shapes = nullptr, *d_steps = nullptr, *d_items = nullptr;
    void *d_entry_pre = nullptr, *d_block_pre = nullptr;
};

namespace sg {

constexpr int kTnThreads = 256;
constexpr int kTnPairsPerThread = 4;   // workspace tables: pair updates per thread and step

// work groups of one workspace table of 2^W entries in a step launch
inline int64_t tn_table_blocks(int W)
{
    const int64_t pairs = W > 0 ? (int64_t{1} << (W - 1)) : 1;
    constexpr int64_t per = int64_t{kTnThreads} * kTnPairsPerThread;
    return (pairs + per - 1) / per;
}

int tn_phase_of(int order, int L, int h, int x, int y, int z);
int tn_n_phases(int order, int L, int h);

}  // namespace sg
