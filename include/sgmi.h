/*
 * sgmi.h -- C ABI of the MI355X (gfx950) annealing library for cubic-lattice
 * Ising spin glasses.
 *
 * The library implements the data-parallel hot path behind the approximate
 * optimisation of Gangat, "Linear-time classical approximate optimization of
 * cubic-lattice classical spin glasses" (arXiv 2501.17267):
 *   - minimise H(s) = sum over nearest-neighbour pairs J_ij s_i s_j over
 *     s in {-1,+1}^N (Sec. I, Eq. 1) on a periodic L x L x L lattice;
 *   - by fixed-sweep-count Metropolis simulated annealing and by parallel
 *     tempering, with or without isoenergetic cluster moves (App. D);
 *   - scored by the optimality gap eps = (E - E_gs)/|E_gs| (Sec. I.A, Eq. 2)
 *     against the exactly known planted ground-state energy of a
 *     tile-planted instance (Sec. II);
 *   - batched over instances of mixed size, served with continuous batching,
 *     and spread over many work-groups for few replicas of large lattices;
 *   - inside the paper's linear-time meta-heuristic (Sec. I), whose
 *     subsystem optimiser is either annealing on l^3 fragments or the exact
 *     tensor-network fragment marginals of App. A-C (and their tropical,
 *     zero-temperature form).
 *
 * Conventions shared by every call
 *   - Lattice: L even, 4 <= L <= SG_MAX_L, N = L^3, site i = x + L*(y + L*z),
 *     periodic in all three directions.  Colour of a site = (x+y+z) mod 2.
 *   - Couplings: int8 J[6][N] in device memory, direction order
 *     +x, -x, +y, -y, +z, -z; J[d][i] couples site i to its d-neighbour, so
 *     each bond is stored twice and the two copies must agree.  Values must
 *     lie in [-4, 4] (sg_check_instance verifies both).
 *   - Spins: int8 +1 / -1, natural site order, [n][N] per call.
 *   - Energies: int32 exact, Eq. 1 with each pair counted once.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed & 0xFFFFFFFF, seed >> 32) and counters
 *       Metropolis proposal at site (x,y,z), colour c, sweep s, replica r:
 *         (col * ceil(L/4) + floor(z/4), 2s + c, r, chain), word z mod 4,
 *         where col = floor(x/2) + (L/2) y;
 *       initial spin of site i of replica r: (floor(i/4), 0xFFFFFFFF, r,
 *         chain), word i mod 4, spin -1 iff the word's top bit is set;
 *       PT exchange of ladder pair k at step t of run `chain`:
 *         (k, t, 0xFFFFFFFF, chain), word 0.
 *     Results depend only on these counters, never on the launch shape.
 *   - Metropolis step (App. D, with the acceptance min(1, exp(-beta dE)) of
 *     the Boltzmann law in App. A): dE = -2 s_i h_i = 2k; k <= 0 always
 *     flips; k > 0 flips iff k <= K and u < thr[row][k-1].  Colour 0 sites
 *     are all updated before colour 1 sites in every sweep.
 *   - Device pointers are borrowed: the library keeps none of them after a
 *     call returns.  The sweep, exchange, energy and gap calls allocate no
 *     device memory; plans, servers and the autotuner allocate theirs when
 *     they are created and free it when they are destroyed.  `stream`
 *     is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *     validate their arguments on the host, enqueue their kernels and return
 *     without waiting for the device.
 *   - Return value: SG_OK (0) or a negative status; sg_last_error() gives a
 *     message for the calling thread.  No C++ exception crosses this ABI.
 */
#ifndef SGMI_H
#define SGMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_OK 0
#define SG_EINVAL (-1)       /* invalid argument (shape, range, null pointer) */
#define SG_ENOMEM (-2)       /* host or device allocation failed */
#define SG_EDEVICE (-3)      /* a HIP runtime call failed */
#define SG_ERANGE (-4)       /* value outside what the tables cover */
#define SG_EBUSY (-5)        /* resource full */
#define SG_ENOTFOUND (-6)    /* unknown handle or request */
#define SG_EUNSUPPORTED (-7) /* valid input the library does not support */

#define SG_MAX_L 64          /* largest lattice the kernels accept */
#define SG_K_MAX 24          /* 6 neighbours x |J| <= 4 */

/* An instance: the couplings of Eq. 1 plus its planted ground-state energy.
 * jenc: optional device buffer of sg_jenc_bytes(L) bytes filled by
 * sg_encode_instance; required for L > SG_LDS_MAX_L (whose couplings are
 * streamed from it during the sweeps), used to speed up the set-up of
 * smaller ones when present.  sa_anneal supports every even L from 4 to
 * 64. */
typedef struct sg_instance {
    int32_t L;
    int32_t reserved;
    const int8_t *J;       /* device int8 [6][L^3] */
    const uint32_t *jenc;  /* device, nullable */
    int64_t E_gs;          /* planted ground-state energy, nonzero */
    uint32_t chain;        /* fourth Philox counter word of this instance's chains */
    uint32_t reserved2;
} sg_instance;

#define SG_LDS_MAX_L 24    /* couplings held in LDS up to this L */

/* Simulated annealing of n_rep independent replicas (App. D: Metropolis
 * sweeps over a beta schedule, one read = the final configuration).
 * Replica r uses Philox counter word rep0 + r.  Sweeps sweep0 ..
 * sweep0+n_sweeps-1 take thr rows 0 .. n_sweeps-1, so a run split into
 * chunks equals the uninterrupted run. */
typedef struct sg_sa_args {
    int32_t n_rep;       /* >= 1 */
    uint32_t rep0;       /* counter word of replica 0 */
    int32_t n_sweeps;    /* >= 1 */
    int32_t sweep0;      /* absolute index of the first sweep, >= 0 */
    int32_t K;           /* row length of thr, 1..SG_K_MAX */
    int32_t init_random; /* 1: draw initial spins from the init stream; 0: use spins[] */
    uint64_t seed;       /* Philox key */
    void *workspace;     /* device scratch of sg_sa_workspace_bytes(L, n_rep) bytes (16-byte
                            aligned) when that is nonzero (L > 32), else ignored */
    int64_t workspace_bytes;
} sg_sa_args;

/* Device scratch an sa_anneal call of lattice size L with n_rep replicas
 * needs (the column-layout spin blocks when a lattice does not fit in LDS):
 * 0 for L <= 32. */
size_t sg_sa_workspace_bytes(int32_t L, int32_t n_rep);

/* thr:    device uint32 [n_sweeps][K] (from sg_make_thresholds)
 * spins:  device int8 [n_rep][N], input when init_random == 0, output always
 * energy: device int32 [n_rep], final energies
 * emin:   device int32 [n_rep] or NULL: lowest energy at the end of a sweep */
int sa_anneal(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr,
              int8_t *spins, int32_t *energy, int32_t *emin, void *stream);

/* Few replicas of a large lattice (even L = 26..64), spread over the
 * whole device.  The method is that of sa_anneal (App. D sweeps, same
 * counters, same result), but each colour phase of each sweep is one
 * launch with one lane per column dword of every replica, instead of one
 * work group per replica group; it cuts the time of one anneal when
 * n_rep is small.  Requires args->workspace of at least
 * n_rep * L^2 * ceil(L/4) * 4 bytes (16-byte aligned), which holds the
 * spins in the column layout; no best-seen energy.  Returns
 * SG_EUNSUPPORTED for other L.
 * sa_anneal takes this path by itself when L > SG_LDS_MAX_L, emin is NULL,
 * the single-work-group kernel selected for L would launch fewer than
 * SG_WIDE_MAX_GROUPS replica groups (so it would leave most compute units
 * idle), and the workspace holds sg_sa_wide_workspace_bytes(L, n_rep)
 * bytes; that function returns 0 when sa_anneal would not take the path. */
#define SG_WIDE_MAX_GROUPS 128
int sg_sa_anneal_wide(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr,
                      int8_t *spins, int32_t *energy, void *stream);
size_t sg_sa_wide_workspace_bytes(int32_t L, int32_t n_rep);

/* Parallel tempering (App. D): n_runs independent runs of T walkers on an
 * ascending beta ladder.  Step t: every walker w makes one sweep with the
 * thresholds of its ladder slot pos[w] (Metropolis counter (., 2t+c, w,
 * run)), then ladder pairs (k, k+1) with k = t mod 2, t mod 2 + 2, ...
 * exchange their walkers with probability
 * min(1, exp(-(beta_{k+1}-beta_k) D)), D = E(walker at k) - E(walker at k+1),
 * i.e. D <= 0 always, else m = D/2 <= M and u < thrx[k][m-1].
 * Run j uses chain = run0 + j as its counter word. */
typedef struct sg_pt_args {
    int32_t n_runs;      /* >= 1 */
    uint32_t run0;
    int32_t T;           /* walkers per run, 2..SG_PT_MAX_T */
    int32_t n_steps;     /* >= 1 */
    int32_t step0;       /* absolute index of the first step, >= 0 */
    int32_t K;           /* row length of thr */
    int32_t M;           /* row length of thrx, >= 1 */
    int32_t init_random; /* 1: init-stream spins and pos[w] = w; 0: use spins[] and pos[] */
    uint64_t seed;
} sg_pt_args;

#define SG_PT_MAX_T 64

/* thr:        device uint32 [T][K], row k = ladder slot k
 * thrx:       device uint32 [T-1][M] (from sg_make_exchange_thresholds)
 * spins:      device int8 [n_runs][T][N] in/out (walker-major)
 * energy:     device int32 [n_runs][T] out
 * pos:        device int32 [n_runs][T] in/out, walker -> ladder slot; with
 *             init_random = 0 a run whose pos is not a permutation of
 *             0..T-1 starts from the identity instead (no LDS index ever
 *             leaves its range)
 * emin_trace: device int32 [n_runs][n_steps] or NULL: min walker energy after each step
 * swap_acc:   device uint32 [n_runs][T-1] or NULL: accepted exchanges per pair, added to */
int pt_run(const sg_instance *inst, const sg_pt_args *args, const uint32_t *thr,
           const uint32_t *thrx, int8_t *spins, int32_t *energy, int32_t *pos,
           int32_t *emin_trace, uint32_t *swap_acc, void *stream);

/* pt_run with each run spread over `groups` work groups (1, 2, 4 or 8; T a
 * multiple of it; 0 picks the most that keep the launch within one work
 * group per compute unit and, unless n_runs is below half the compute
 * units, give each group at least 512 of the T*L^2/2 column units of a
 * colour phase; with fewer runs it splits only when T*L^3 >= 6144, and
 * returns 1 when nothing qualifies), for fewer runs than the device has compute
 * units: group g sweeps walkers g*T/groups .. (g+1)*T/groups - 1, and the
 * groups of a run pass their walkers' energies to each other through the
 * workspace once per step, then make the same exchange decisions.  Results
 * are identical to pt_run's, bit for bit.  waves: waves per work group (0,
 * 4, 8, 12, 16; 0 picks).  workspace: device memory of
 * sg_pt_split_workspace_bytes(n_runs, T) bytes, 8-byte aligned, owned by the
 * caller; may be NULL only with groups = 1.  The call clears it on the
 * stream first; its first int32 is a status read after the call completes:
 * 0, or bit 0 set if a group gave up waiting on another (a group waits at
 * most a few seconds; the results are then invalid), bit 1 set if a run's
 * pos was not a permutation (the identity was used).  Calls sharing one
 * workspace must not overlap.
 * SG_EUNSUPPORTED when the launch's work groups would not all be resident on
 * the device at once. */
int sg_pt_run_split(const sg_instance *inst, const sg_pt_args *args, int32_t groups, int32_t waves,
                    const uint32_t *thr, const uint32_t *thrx, int8_t *spins, int32_t *energy,
                    int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc, void *workspace,
                    int64_t workspace_bytes, void *stream);
size_t sg_pt_split_workspace_bytes(int32_t n_runs, int32_t T);

/* sg_pt_run_split without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation).  The mailbox lives
 * in a fixed device array of SG_PT_STATIC_SCRATCH_BYTES bytes inside the
 * library (one per GPU, held until the process ends), so calls with
 * sg_pt_split_workspace_bytes(n_runs, T) above that size return SG_ERANGE.
 * Every other argument, the group choice and the results are those of
 * sg_pt_run_split.  status_out: device int32 or NULL; after the call
 * completes it holds the status word of sg_pt_run_split (0: no problem).  The call clears the array's mailbox on the
 * stream before its kernel.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (other streams, other threads) race and
 * must not be issued. */
#define SG_PT_STATIC_SCRATCH_BYTES (1 << 20)
int sg_pt_run_split_static(const sg_instance *inst, const sg_pt_args *args, int32_t groups, int32_t waves,
                           const uint32_t *thr, const uint32_t *thrx, int8_t *spins, int32_t *energy,
                           int32_t *pos, int32_t *emin_trace, uint32_t *swap_acc, int32_t *status_out,
                           void *stream);

/* ---- parallel tempering with isoenergetic cluster moves (App. D, PT+ICM) ----
 * The paper only names the cluster moves; this is Houdayer's two-replica
 * move as combined with PT by Zhu, Ochoa and Katzgraber (2015).  Two copies
 * of a T-slot ladder: walkers w = 0..2T-1, copy(w) = w / T (fixed), pos[w]
 * = slot of w inside its copy.  Step t:
 *   1. every walker makes one sweep (thresholds row pos[w], Metropolis
 *      counter (., 2t+c, w, run), as pt_run);
 *   2. for slots k = icm_from .. T-1, with a, b the walkers of copy 0 and 1
 *      at slot k: the sites where they differ are ordered by (colour,
 *      column, height) of the column layout (colour (x+y+z) mod 2, column
 *      x/2 + (L/2) y, height z); if there are n > 0, the seed is number
 *      floor(u n / 2^32), u = Philox word 0 of (k, t, 0xFFFFFFFE, run); the
 *      cluster is every differing site connected to the seed through
 *      differing sites and nonzero couplings; both walkers flip it (their
 *      summed energy is unchanged, so the move is always taken);
 *   3. inside each copy cp, ladder pairs (k, k+1), k = t mod 2, ... exchange
 *      as in pt_run with u = Philox word 0 of (k + cp T, t, 0xFFFFFFFF, run).
 * With icm_from >= T, copy 0 is exactly pt_run's chain. */
#define SG_PTICM_MAX_T 32
typedef struct sg_pticm_args {
    int32_t n_runs;      /* >= 1 */
    uint32_t run0;
    int32_t T;           /* slots per copy, 2..SG_PTICM_MAX_T (2T walkers) */
    int32_t n_steps;     /* >= 1 */
    int32_t step0;       /* absolute index of the first step, >= 0 */
    int32_t K;           /* row length of thr */
    int32_t M;           /* row length of thrx, >= 1 */
    int32_t init_random; /* 1: init-stream spins (replica word w) and pos[w] = w mod T */
    int32_t icm_from;    /* first slot with cluster moves (>= T: none) */
    int32_t reserved;
    uint64_t seed;
} sg_pticm_args;

/* thr [T][K], thrx [T-1][M] as pt_run; spins [n_runs][2T][N], energy
 * [n_runs][2T], pos [n_runs][2T] in/out; emin_trace [n_runs][n_steps]
 * (minimum over the 2T walkers after each step), swap_acc [n_runs][2(T-1)]
 * (copy-major, added to) and icm_flipped [n_runs][n_steps] (sites flipped
 * per walker by the step's cluster moves) are nullable.  L <= 16. */
int sg_pticm_run(const sg_instance *inst, const sg_pticm_args *args, const uint32_t *thr,
                 const uint32_t *thrx, int8_t *spins, int32_t *energy, int32_t *pos,
                 int32_t *emin_trace, uint32_t *swap_acc, int32_t *icm_flipped, void *stream);

/* ---- the linear-time meta-heuristic (Sec. I) with simulated annealing as the
 * subsystem optimiser, bootstrapped over overlapping fragments (App. C) ----
 * The lattice is tiled by cores of c^3 spins (L % c == 0, nb = L/c per axis,
 * core k = bx + nb (by + nb bz)); the fragment of a core is the l^3 cube,
 * l = c + 2h, that extends it by h sites on every side (periodic).  Cores
 * are decimated phase by phase; all cores of a phase run at once and see
 * the decimation state at the start of their phase:
 *   order 0: phase (bx mod P) + P((by mod P) + P(bz mod P)), P = 1 +
 *            ceil(h/c), nb % P == 0 (colour classes: no core of a phase lies
 *            in another's fragment);
 *   order 1: phase bx + by + bz (a diagonal wavefront: each core sees the
 *            decimated cores below it).
 * A core is processed by R independent anneals of its fragment.  Site j =
 * lx + l (ly + l lz) is fixed (a boundary field) when it was decimated in
 * an earlier phase, else free; only bonds with both ends in the fragment
 * count.  Anneal r starts its free spins from bit 31 of Philox word 0 of
 * (r l^3 + j, 0xFFFFFFFF, k, run) (set: -1) and makes n_sweeps sweeps
 * (colour (x+y+z) mod 2 = 0, then 1) of Metropolis proposals at its free
 * sites with u = Philox word s mod 4 of (r l^3 + j, 2 floor(s/4) + colour,
 * k, run) (one call serves a site's four sweeps 4m..4m+3) against thr row s
 * (as sa_anneal).  The anneal with the lowest in-fragment energy
 * (lowest r among equals) gives the core's spins.  The time is linear in
 * N: N/c^3 fragments of fixed cost. */
#define SG_FRAG_MAX_L 9      /* largest fragment edge l */
#define SG_FRAG_MAX_R 16     /* most anneals per fragment */
typedef struct sg_frag_args {
    int32_t core;       /* c >= 1, divides L */
    int32_t halo;       /* h >= 0; l = c + 2h < L and <= SG_FRAG_MAX_L */
    int32_t replicas;   /* R anneals per fragment, 1..SG_FRAG_MAX_R */
    int32_t order;      /* 0 colour classes, 1 diagonal wavefront */
    int32_t n_runs;     /* independent decimations; run j uses counter word run0 + j */
    uint32_t run0;
    int32_t n_sweeps;   /* sweeps per fragment anneal = rows of thr */
    int32_t K;          /* row length of thr, 1..SG_K_MAX */
    uint64_t seed;      /* Philox key */
} sg_frag_args;

/* inst->J (natural order) is required.  thr: device uint32 [n_sweeps][K];
 * spins_out: device int8 [n_runs][N], the decimated configurations (+-1);
 * energy_out: device int32 [n_runs] or NULL, their energies (Eq. 1).
 * SG_EINVAL for shapes outside the rules above, SG_ERANGE when the run
 * counter words overflow or n_runs * nb^3 exceeds one launch. */
int sg_fragment_decimate(const sg_instance *inst, const sg_frag_args *args, const uint32_t *thr,
                         int8_t *spins_out, int32_t *energy_out, void *stream);

/* ---- tensor-network fragment decimation (Sec. I, App. A-C) ----------------
 * The paper's own subsystem optimiser: single-spin decimation from the
 * exact marginal of a fragment.  The fragment of site i is the l^3 cube,
 * l = 2h + 1, centred on i (periodic wrap, l < L); only bonds with both
 * ends in the cube belong to it.  Sites are decimated phase by phase,
 *   order 0: phase (x mod P) + P((y mod P) + P(z mod P)), P = 1 + h,
 *            L % P == 0 (no two sites of a phase share a fragment);
 *   order 1: phase x + y + z (diagonal wavefront).
 * A fragment site decimated in an earlier phase is fixed at its value, the
 * others are free (every site of a phase sees the state at the phase's
 * start).  With Z(s) = sum over the free spins other than i of
 * exp(-beta E_frag), E_frag the fragment's share of Eq. 1 with s_i = s,
 * site i takes +1 when ln Z(+1) >= ln Z(-1), else -1 (its most probable
 * value).  The tropical form (the zero-temperature variant named in
 * Sec. III) uses the least fragment energy E(s) instead: +1 when
 * E(+1) <= E(-1).  The contraction is exact (no truncation): each
 * fragment's free spins are summed out one by one over a table indexed by
 * the spins still connected to the summed part.
 *
 * A plan holds what depends only on (L, h, order): the distinct fragment
 * shapes and the elimination program of each.  Tables of at most
 * 2^lds_max_bits entries are contracted in LDS by one work group; larger
 * ones live in the caller's workspace (at most 2^SG_TN_MAX_BITS entries).
 */
#define SG_TN_MAX_HALO 2     /* l = 2h + 1 <= 5, the paper's fragment edge */
#define SG_TN_MAX_BITS 26    /* largest elimination table: 2^26 doubles */
#define SG_TN_LDS_BITS 13    /* default LDS tier: tables of up to 2^13 entries */
typedef struct sg_tn_plan sg_tn_plan;

typedef struct sg_tn_plan_info {
    int32_t L, halo, order, lds_max_bits;
    int32_t n_phases;
    int32_t n_shapes;            /* distinct free-site patterns */
    int32_t max_bits;            /* largest table, log2 entries */
    int32_t n_lds_sites;         /* sites contracted in LDS */
    int32_t n_hbm_sites;         /* sites contracted in the workspace */
    int32_t max_steps;           /* most eliminations of one fragment */
    double pair_updates;         /* table pair updates per decimation (both values of s_i) */
} sg_tn_plan_info;

/* Plan the decimation of an L^3 lattice with fragment halo h (1..SG_TN_MAX_HALO)
 * in phase order `order`.  lds_max_bits: the largest table contracted in LDS
 * (0 = SG_TN_LDS_BITS; 1..SG_TN_LDS_BITS).  Host work only: the plan's
 * tables go to the device on its first decimation and stay there until
 * sg_tn_plan_destroy; a plan serves the device current at that call.
 * SG_EINVAL for shapes outside the rules above, SG_EUNSUPPORTED when a
 * fragment would need a table above 2^SG_TN_MAX_BITS. */
int sg_tn_plan_create(int32_t L, int32_t halo, int32_t order, int32_t lds_max_bits, sg_tn_plan **out);
int sg_tn_plan_info_get(const sg_tn_plan *plan, sg_tn_plan_info *out);
int sg_tn_plan_destroy(sg_tn_plan *plan);

/* The plan's elimination programs, for inspection (host memory; any
 * pointer may be NULL to skip that array; the counts are always written):
 *   shapes [n_shapes][4]: table bits W, step count, first step, and a 6-bit
 *     mask of the centre's neighbour directions that are fixed sites;
 *   steps [n_steps][16]: eliminated local site j = lx + l (ly + l lz), its
 *     table slot a, then per direction +x,-x,+y,-y,+z,-z the neighbour's
 *     code: its slot (>= 0), -1 fixed, -2 the centre, -3 outside or
 *     eliminated; then the workspace tier's canonical-entry bookkeeping:
 *     whether slot a was active before the step, the number of runs of
 *     consecutive canonical slots other than a, their total length, the
 *     mask of slots that become active at the step (a excluded), and the
 *     runs packed four to an int: byte r%4 of int 12 + r/4 = start of run
 *     r, of int 14 + r/4 = its length;
 *   items [N][2]: every site as (centre site, shape), phase by phase. */
int sg_tn_plan_program(const sg_tn_plan *plan, int32_t *n_shapes, int32_t *shapes, int32_t *n_steps,
                       int32_t *steps, int32_t *n_items, int32_t *items);

/* The plan's rounds, for inspection (host memory; either array may be NULL,
 * the count is always written).  A round is one step of a shape or two
 * consecutive ones that the workspace tier runs in one pass over the table
 * (sum-product tables are renormalised after each round, in both tiers):
 *   shape_rounds [n_shapes][2]: the shape's first round and round count;
 *   rounds [n_rounds][4]: the first step (within its shape), 1 when the
 *     round also runs the next step, the canonical read bits of the round
 *     (assignments read = 2^bits), and the case of the second step's slot b
 *     (0: b takes its slot at that step, 1: b is canonical at the first
 *     step, 2: b becomes active at the first step) | b's rank among the
 *     first step's canonical bits << 8.
 * Pairs run fused only when beta <= SG_TN_FUSE_BETA_MAX or in the tropical
 * form; otherwise every step is its own round. */
#define SG_TN_FUSE_BETA_MAX 9.5
int sg_tn_plan_rounds(const sg_tn_plan *plan, int32_t *n_rounds, int32_t *shape_rounds, int32_t *rounds);

/* Workspace for n_inst instances: `full` = 0 gives the least that works
 * (the workspace tables are then processed in several passes), 1 the size
 * that holds the largest phase of all instances at once. */
int64_t sg_tn_workspace_bytes(const sg_tn_plan *plan, int32_t n_inst, int32_t full);

typedef struct sg_tn_args {
    const int8_t *J;     /* device int8 [n_inst][6][N], values in [-4, 4] */
    int32_t n_inst;      /* instances of the plan's L decimated together */
    int32_t tropical;    /* 1: min-plus form (beta unused) */
    double beta;         /* inverse temperature, 0 < beta <= 14 (no overflow for |h| <= 24) */
    int8_t *spins_out;   /* device int8 [n_inst][N]: the decimated spins */
    double *score_out;   /* device double [n_inst][N] or NULL: each site's
                            ln Z(+1) - ln Z(-1), or E(-1) - E(+1) when tropical */
    int32_t *energy_out; /* device int32 [n_inst] or NULL: Eq. 1 of spins_out */
    void *workspace;     /* device, workspace_bytes >= sg_tn_workspace_bytes(plan, n_inst, 0) */
    int64_t workspace_bytes;
} sg_tn_args;

/* Decimate n_inst instances with the plan.  SG_EINVAL for bad arguments
 * (including a workspace below the minimum), SG_ERANGE when 2 n_inst times
 * the sites of a phase exceeds one launch (2^31 work groups), SG_ENOMEM
 * when the plan's first upload fails.  Part of the work runs on two streams the plan owns,
 * forked from `stream` and joined back to it within the call's work, so
 * everything stays ordered with respect to `stream`; calls with one plan
 * must not overlap (they share those streams), and the plan must outlive them. */
int sg_tn_decimate(sg_tn_plan *plan, const sg_tn_args *args, void *stream);

/* Energy (Eq. 1) of n_rep configurations spins [n_rep][N] -> energy [n_rep]. */
int energy(const sg_instance *inst, int32_t n_rep, const int8_t *spins, int32_t *energy_out,
           void *stream);

/* Optimality gap (Eq. 2): eps[i] = (energy[i] - E_gs) / |E_gs| in double,
 * from exact integers.  energy and eps_out are device arrays of n entries. */
int epsilon(const int32_t *energy, int64_t n, int64_t E_gs, double *eps_out, void *stream);

/* Optimality-gap statistics per instance (Eq. 2, and the TT-eps criterion
 * of App. D: a target is reached when the mean gap over an instance's
 * trials is at or below it).  energy: device int32 [n_groups][group_size],
 * the trials of group g contiguous; E_gs: device int64 [n_groups], nonzero.
 * With eps_i = (E_i - E_gs[g]) / |E_gs[g]| in double from exact integers
 * (as epsilon()), stats_out[g] (device) receives the exact energy sum (so
 * the mean gap is (sum - n E_gs) / (n |E_gs|)), the least and greatest
 * energy, and n_le[t] = the number of trials with eps_i <= targets[t] for
 * the n_targets (0..SG_EPS_MAX_TARGETS) host values targets[].  hist_out
 * (device uint32 [n_groups][n_bins], nullable; n_bins 1..SG_EPS_MAX_BINS,
 * eps_max > 0) counts the trials per bin floor(eps_i / eps_max * n_bins),
 * negative gaps in bin 0 and gaps at or above eps_max in bin n_bins-1.
 * One work group per group; the outputs are overwritten, not added to.
 * SG_EINVAL for bad shapes or pointers; an E_gs entry of 0 gives a
 * division by zero (inf/nan gaps), not an error, since E_gs is not read on
 * the host. */
#define SG_EPS_MAX_TARGETS 8
#define SG_EPS_MAX_BINS 1024
typedef struct sg_eps_stats {
    int64_t energy_sum;
    int32_t energy_min;
    int32_t energy_max;
    int32_t n;                           /* group_size */
    int32_t n_le[SG_EPS_MAX_TARGETS];    /* entries past n_targets are 0 */
    int32_t reserved;
} sg_eps_stats;

int epsilon_stats(const int32_t *energy, int32_t n_groups, int32_t group_size, const int64_t *E_gs,
                  const double *targets, int32_t n_targets, double eps_max, int32_t n_bins,
                  sg_eps_stats *stats_out, uint32_t *hist_out, void *stream);

/* ---- launch shapes and autotuning -----------------------------------------------
 * The annealing kernel exists in several launch shapes per lattice size
 * ("variants": replicas per work group, waves per work group, whether LDS
 * holds both coupling encodings).  All produce bit-identical results; they
 * differ only in speed.  sa_anneal and new batch plans use the selected
 * variant of each size (the first one until a selection or autotune). */
typedef struct sg_sa_variant {
    int32_t L;
    int32_t replicas_per_group;
    int32_t waves_per_group;
    int32_t both_encodings;   /* 1: E and F coupling encodings; 0: E only */
    int32_t couplings_in_hbm; /* 1: couplings streamed from the encoded buffer */
    int32_t spins_in_hbm;     /* 1: spins in the workspace instead of LDS */
    int32_t reserved;
    int64_t lds_bytes;        /* LDS per work group */
} sg_sa_variant;

typedef struct sg_sa_tune_result {
    int32_t variant;
    int32_t identical;        /* 1 if its output equalled variant 0's bit for bit */
    float ms;                 /* mean device time of one call */
    double attempts_per_s;
} sg_sa_tune_result;

/* Writes up to max variants of size L into out; returns the count. */
int sg_sa_variants(int32_t L, int32_t max, sg_sa_variant *out);
int sg_sa_select_variant(int32_t L, int32_t variant);
/* selected variant index of size L (or a negative status) */
int sg_sa_selected_variant(int32_t L);
/* sa_anneal with an explicit variant */
int sg_sa_anneal_variant(const sg_instance *inst, const sg_sa_args *args, const uint32_t *thr,
                         int8_t *spins, int32_t *energy, int32_t *emin, int32_t variant,
                         void *stream);
/* Autotuner: anneals one synthetic instance of size L (n_rep replicas,
 * n_sweeps sweeps, beta linear 0.1 -> 3.0) with every variant, `repeats`
 * timed calls each, checks that all outputs are bit-identical, selects the
 * fastest and returns its index.  Fills out[0..max_out) with the timings.
 * Allocates and frees its own device buffers; synchronous. */
int sg_autotune_sa(int32_t L, int32_t n_rep, int32_t n_sweeps, int32_t repeats,
                   sg_sa_tune_result *out, int32_t max_out, void *stream);

/* ---- batched annealing ----------------------------------------------------------
 * Many sa_anneal calls (instances of different L, replica counts and sweep
 * budgets) fused into one schedule.  Each job keeps exactly the semantics
 * of the sa_anneal call it describes: results are bit-identical to running
 * the jobs one by one, in any order.  The plan groups jobs by L, orders each
 * group's work longest first, uploads the job tables to device memory it
 * owns, and launches one kernel per L on parallel branches; with
 * SG_BATCH_GRAPH the whole schedule is captured once as a hipGraph and each
 * sg_batch_launch replays it.  A plan stores the jobs' device pointers:
 * they must stay valid while the plan is launched. */
typedef struct sg_sa_job {
    sg_instance inst;
    sg_sa_args args;
    const uint32_t *thr;   /* device [n_sweeps][K] */
    int8_t *spins;         /* device [n_rep][N] */
    int32_t *energy;       /* device [n_rep] */
    int32_t *emin;         /* device [n_rep] or NULL */
} sg_sa_job;

typedef struct sg_batch sg_batch;

#define SG_BATCH_GRAPH 1   /* capture the schedule as a hipGraph */

int sg_batch_create(const sg_sa_job *jobs, int32_t n_jobs, int32_t flags, sg_batch **out);
int sg_batch_launch(sg_batch *batch, void *stream);
/* n_kernels: kernels per launch; attempts: spin-flip attempts per launch */
int sg_batch_info(const sg_batch *batch, int32_t *n_kernels, int64_t *n_groups, double *attempts);
/* Per-kernel view of the plan, one entry per lattice size (up to n):
 * L, spin-flip attempts per launch, and the device time in ms of that
 * kernel in the most recent completed launch (-1 if unavailable).
 * Returns the number of entries written. */
int sg_batch_kernels(const sg_batch *batch, int32_t n, int32_t *L_out, double *attempts_out,
                     float *ms_out);
/* waits for the plan's work to finish, then frees it */
int sg_batch_destroy(sg_batch *batch);

/* ---- serving: continuous batching of anneal requests ---------------------------
 * A request anneals one replica of an instance for n_sweeps sweeps with its
 * own schedule rows, seed and replica counter word.  A server thread admits
 * queued requests, in arrival order but passing over (for a bounded time)
 * one that does not fit yet, while the active limit, the memory budget
 * (request state: spins + energy + workspace) and the pool of large-lattice
 * workspaces allow, and advances all active requests in chunks of chunk_sweeps: each
 * lattice size has its own stream, and every time a size's previous chunk
 * finishes, all its active requests -- including those admitted meanwhile --
 * run their next chunk together in one kernel.  A request's result depends
 * only on its own content (instance, schedule, seed, replica word), never on
 * the mix, the slot or the chunking: it equals one sa_anneal call.
 * The server allocates its own device memory (job tables, workspace pool)
 * at creation and when a lattice size first appears; it borrows the request
 * arrays until the request is done or cancelled. */
typedef struct sg_server_config {
    int32_t max_active;      /* requests on the device at once (0: 4096) */
    int32_t chunk_sweeps;    /* most sweeps per request per chunk (0: 64) */
    int64_t memory_budget;   /* bytes of admitted request state (0: 8 GiB) */
    int32_t large_slots;     /* preallocated workspaces for lattices above L = 32 */
    int32_t skip_age_ms;     /* a queued request that does not fit is passed over by later
                                ones while it is younger than this (0: 50 ms); older, it
                                holds back everything queued after it until it fits */
    int64_t chunk_attempts;  /* > 0: a size's chunk is max(1, min(chunk_sweeps,
                                chunk_attempts / L^3)) sweeps, so chunks of all sizes
                                take similar time; 0: chunk_sweeps for every size */
} sg_server_config;

typedef struct sg_request {
    sg_instance inst;        /* couplings must stay valid until the request ends */
    const uint32_t *thr;     /* device [n_sweeps][K] */
    int32_t n_sweeps;
    int32_t K;
    uint64_t seed;           /* Philox key */
    uint32_t replica;        /* Philox replica counter word */
    int32_t init_random;     /* 1: init stream; 0: start from spins[] */
    int8_t *spins;           /* device [N], in/out; final configuration when done */
    int32_t *energy;         /* device [1]: energy after the latest chunk */
    double t_arrival;        /* arrival time on the server clock, for latency */
} sg_request;

#define SG_REQ_QUEUED 0
#define SG_REQ_ACTIVE 1
#define SG_REQ_DONE 2
#define SG_REQ_CANCELLED 3
#define SG_REQ_FAILED 4

typedef struct sg_request_status {
    int32_t state;           /* SG_REQ_* */
    int32_t done_sweeps;
    double t_arrival, t_admit, t_done;   /* server clock, seconds */
} sg_request_status;

typedef struct sg_server_stats {
    int64_t submitted, completed, cancelled, active, queued, launches;
    double attempts_completed;
    int64_t memory_in_use;
} sg_server_stats;

typedef struct sg_server sg_server;

int sg_server_create(const sg_server_config *cfg, sg_server **out);
double sg_server_now(const sg_server *srv);          /* server clock (steady, seconds) */
int sg_server_submit(sg_server *srv, const sg_request *req, uint64_t *id_out);
/* SG_OK with the request's status, SG_ENOTFOUND for an unknown id */
int sg_server_poll(sg_server *srv, uint64_t id, sg_request_status *out);
/* queued: dropped at once; active: retired at its next chunk boundary */
int sg_server_cancel(sg_server *srv, uint64_t id);
/* forget a finished (done, cancelled or failed) request: its id becomes
 * unknown and the server's record of it is freed; SG_EBUSY while it is
 * queued or active.  A long-running server's callers release every request
 * once they have read its result. */
int sg_server_release(sg_server *srv, uint64_t id);
int sg_server_get_stats(sg_server *srv, sg_server_stats *out);
/* blocks until no request is queued or active (SG_EBUSY on timeout) */
int sg_server_wait(sg_server *srv, double timeout_s);
/* cancels what is left, waits for the device, frees the server */
int sg_server_destroy(sg_server *srv);

/* ---- host helpers (synchronous, no device work) ---------------------------- */

const char *sg_strerror(int code);
const char *sg_last_error(void);   /* thread-local message of the last failure */
const char *sg_version(void);

/* beta schedule: kind 0 linear b0 + (b1-b0) s/(S-1); kind 1 geometric
 * b0 (b1/b0)^(s/(S-1)); S == 1 gives b0.  beta_out: host double [S]. */
int sg_make_schedule(int32_t kind, double b0, double b1, int32_t S, double *beta_out);

/* Metropolis table: thr_out[s][k-1] = min(2^32-1, floor(exp(-(2k) beta_s) 2^32)),
 * k = 1..K.  Host arrays beta [S], thr_out [S][K]. */
int sg_make_thresholds(const double *beta, int32_t S, int32_t K, uint32_t *thr_out);

/* Exchange table: thrx_out[k][m-1] = min(2^32-1, floor(exp(-(2m)(beta_{k+1}-beta_k)) 2^32)),
 * m = 1..M.  Host arrays beta [T], thrx_out [T-1][M]. */
int sg_make_exchange_thresholds(const double *beta, int32_t T, int32_t M, uint32_t *thrx_out);

/* Smallest M for which the exchange table of the ladder has no nonzero
 * entry cut off (the table is zero beyond). */
int32_t sg_exchange_table_width(const double *beta, int32_t T);

/* Synthetic tile-planted instance (a stand-in for the tile-planting model of
 * Sec. II): unit cubes with even lower-corner parity are tiles; each draws
 * twelve couplings in {-2,-1,1,2} until it has `cls` frustrated faces
 * (cls in {0,2,4,6}; -1 = any); each tile is gauged so that all +1 is one
 * of its ground states; bonds sum their two tiles; a random gauge hides
 * the planted state.  Host outputs J [6][N], planted [N] (+-1), E_gs. */
int sg_make_instance(int32_t L, int32_t cls, uint64_t seed, int8_t *J_host,
                     int8_t *planted_host, int64_t *E_gs);

/* ---- device helpers ------------------------------------------------------------ */

/* Bytes of the encoded-coupling buffer used by the kernels for lattice L. */
size_t sg_jenc_bytes(int32_t L);

/* Fill inst->jenc-sized device buffer `jenc_out` from inst->J. */
int sg_encode_instance(const sg_instance *inst, uint32_t *jenc_out, void *stream);

/* Validate inst->J on the device: *status_out (device int32) receives 0 if
 * every coupling lies in [-4, 4] and the two copies of every bond agree,
 * otherwise 1 + the number of offending entries (saturating). */
int sg_check_instance(const sg_instance *inst, int32_t *status_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
