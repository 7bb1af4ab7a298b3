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

// The workspace tier updates only "canonical" entries, those whose bits
// of free slots are 0 (the other entries are copies of them).  Before step t
// the canonical bits are the slots P active after step t-1.  The step reads,
// for every assignment of P minus the eliminated slot a, the entries with
// a = 0 and a = 1 (one entry when v only now takes its slot: the table is
// constant along a), and writes every combination of the slots that become
// active at this step ("new", a excluded), with a = 0.  No thread reads a
// location another thread writes, so the update is in place.
struct TnStep {
    int16_t lv;        // local index of the eliminated spin, lx + l (ly + l lz)
    uint8_t a;         // its slot
    uint8_t a_active;  // 1 when slot a was already active before the step
    int8_t code[6];    // per direction +x,-x,+y,-y,+z,-z: slot (>= 0) or kTn*
    uint8_t n_runs;    // canonical bits other than a as runs of consecutive slots
    uint8_t n_base;    //   and their count
    uint32_t newmask;  // slots that become active at this step, a excluded
    uint8_t run_start[8];
    uint8_t run_len[8];
};
static_assert(sizeof(TnStep) == 32, "TnStep layout");

// A round is one step, or two consecutive steps t, t + 1 ("fused") that
// the workspace tier runs in one pass: every assignment of the canonical
// slots of step t other than the slot b of step t + 1 reads its entries
// (a and b = 0, 1 where active), applies step t to them in registers, then
// step t + 1, and writes only step t + 1's entries.  Sum-product tables are
// renormalised after each round (so both tiers renormalise there).  Steps
// are paired greedily from the first; a pair is fused when step t + 1 is not
// the last step and step t leaves at most kTnFuseMax values per read
// assignment (2^|new slots of t|, twice that when b is canonical at t).
constexpr int kTnFuseMax = 8;

struct TnRound {
    int16_t step;      // first step, within its shape
    uint8_t fused;     // 1: also runs step + 1
    uint8_t read_bits; // canonical read bits of the round (bits of p per read assignment)
    uint8_t b_mode;    // slot b of step + 1: 0 new at step + 1, 1 canonical at step, 2 new at step
    uint8_t b_rank;    //   its rank among step's canonical bits (mode 1)
    uint8_t pad[2];
};
static_assert(sizeof(TnRound) == 8, "TnRound layout");

struct TnShape {
    int32_t W;         // table bits (2^W entries)
    int32_t n_steps;   // eliminations
    int32_t step0;     // first step in the step array
    int8_t ccode[6];   // the centre's neighbours: kTnConst (fixed) or kTnNone
    int16_t max_base;  // most canonical read bits of a step (workspace tier)
    int32_t round0;    // first round in the round array
    int32_t n_rounds;
};
static_assert(sizeof(TnShape) == 28, "TnShape layout");

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
    std::vector<sg::TnRound> rounds;
    std::vector<sg::TnItem> items;
    std::vector<sg::TnPhase> phases;
    // workspace items in phase order: table-entry prefix of one instance
    // (both centre values), per phase relative to the phase start
    std::vector<int64_t> hbm_entry_pre;   // [n_hbm_total + n_phases]
    int32_t max_bits = 0, max_steps = 0, n_lds = 0, n_hbm = 0, max_items = 0;
    double pair_updates = 0;
    // device copies (first decimation)
    std::mutex mu;
    int device = -1;
    void *d_shapes = nullptr, *d_steps = nullptr, *d_rounds = nullptr, *d_items = nullptr;
    void *d_entry_pre = nullptr;
    // the LDS tier runs beside the workspace tier on a stream of the plan
    // (default priority), forked from and joined to the caller's stream
    void *side = nullptr, *fork = nullptr, *join = nullptr;   // hipStream_t, hipEvent_t x 2
    // the second half of a workspace-tier batch's instances runs on a
    // second stream of the plan, so that one half's next step can fill the
    // device while the other half's step drains
    void *side2 = nullptr, *fork2 = nullptr, *join2 = nullptr;
};

namespace sg {

constexpr int kTnThreads = 256;
constexpr int kTnReadsInFlight = 4;    // workspace tables: canonical reads a thread issues at once
constexpr int kTnPairsPerThread = 4;   //   and reads per thread and step (in rounds of the above)

// work groups per workspace table in a step launch: enough for 2^n_base
// canonical reads, kTnPairsPerThread per thread
inline int64_t tn_table_blocks(int n_base)
{
    const int64_t items = int64_t{1} << n_base;
    constexpr int64_t per = int64_t{kTnThreads} * kTnPairsPerThread;
    return (items + per - 1) / per;
}

int tn_phase_of(int order, int L, int h, int x, int y, int z);
int tn_n_phases(int order, int L, int h);

}  // namespace sg
