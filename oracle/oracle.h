/*
 * oracle.h -- plain, slow, single-threaded C reference for the annealing hot
 * path of "Linear-time classical approximate optimization of cubic-lattice
 * classical spin glasses" (Gangat, arXiv 2501.17267).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the HIP
 * path: every definition below is written out again, from the paper and the
 * published definitions of Philox4x32-10 and splitmix64, in the most direct
 * form.
 *
 * What is computed, and where the paper fixes it:
 *   energy      Eq. (1), H = sum over nearest-neighbour pairs J_ij s_i s_j
 *   epsilon     Eq. (2), eps = (E - E_gs)/|E_gs|
 *   sa_run      App. D (Simulated Annealing): Metropolis sweeps over a
 *               beta schedule, one read = the final configuration
 *   pt_run      App. D (Parallel Tempering): Metropolis sweeps of T walkers
 *               on a ladder of betas plus neighbour replica exchange
 *   pticm_run   App. D (PT with isoenergetic cluster moves): two copies of
 *               the ladder plus a cluster move between them per slot
 *   make_inst   Sec. II: tile-planted instance with a gauge-scrambled
 *               planted ground state and exactly known E_gs (synthetic
 *               stand-in: the tile classes of the paper are defined only
 *               in its references)
 *   Boltzmann   App. A: the target law p(s) ~ exp(-beta H(s)) that fixes
 *               the Metropolis acceptance min(1, exp(-beta dE))
 *   frag_*      Sec. I and App. C: the bootstrapped subsystem-optimisation
 *               meta-heuristic, with fixed-sweep simulated annealing as the
 *               subsystem optimiser on overlapping cubic fragments
 *
 * Parity pins for every function live in tests/test_oracle_*.py.  One part
 * is "parity unpinned": the 64-bit finaliser of orc_sm64_next (its
 * multipliers and shifts).  No published known-answer output of splitmix64
 * is available to test it against, and the Weyl-sequence test holds for any
 * finaliser.  A wrong finaliser would change which stand-in instance a seed
 * draws, not whether the instance is valid: the planting, class and
 * brute-force pins check validity for whatever stream is drawn.
 *
 * The conventions fixed here (counter layouts, seed orders, phase orders)
 * are frozen: a change to them names the reading it follows and adds a pin.
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- lattice -------------------------------------------------------------
 * Box Lx x Ly x Lz, site i = x + Lx*(y + Ly*z).  Directions d = 0..5 are
 * +x, -x, +y, -y, +z, -z.  Neighbours wrap periodically; an open box is a
 * periodic one whose wrap-around couplings are zero.
 * J is int8 [6][N]: J[d*N + i] couples site i to its d-neighbour, so each
 * bond appears twice (J[+x][i] == J[-x][i+x] and so on). */
int64_t orc_site(int Lx, int Ly, int Lz, int x, int y, int z);
int64_t orc_nbr(int Lx, int Ly, int Lz, int64_t i, int d);

/* ---- splitmix64 (Steele, Lea, Flood 2014) -------------------------------- */
uint64_t orc_sm64_next(uint64_t *state);

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -------------------
 * out[0..3] = Philox4x32_10(counter ctr[0..3], key (k0, k1)). */
void orc_philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]);

/* ---- instance generator (synthetic tile planting) ------------------------
 * cls = number of frustrated faces every tile must have (0, 2, 4 or 6);
 * -1 = no face filter.  periodic = 1 for a periodic box (all dims even),
 * 0 for an open box.  Writes J[6][N], planted[N] (+1/-1) and E_gs. */
int orc_make_instance(int Lx, int Ly, int Lz, int periodic, int cls, uint64_t seed,
                      int8_t *J, int8_t *planted, int64_t *E_gs);

/* ---- energy and optimality gap ------------------------------------------ */
int64_t orc_energy(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *s);
int64_t orc_local_field(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *s, int64_t i);
double  orc_epsilon(int64_t E, int64_t E_gs);

/* ---- optimality-gap statistics (Eq. 2; App. D's TT-eps criterion) ---------
 * Groups g = 0..n_groups-1 of group_size consecutive energies (the trials of
 * one instance).  For each group, with eps_i = orc_epsilon(E_i, E_gs[g]):
 *   sum[g]   exact sum of the energies (the mean eps over the group is then
 *            (sum - n E_gs) / (n |E_gs|), one division);
 *   emin[g], emax[g]  least and greatest energy;
 *   n_le[g*n_targets + t]  how many eps_i <= targets[t];
 *   hist[g*n_bins + b]     how many eps_i fall in bin b, where the bin of eps
 *            is floor(eps / eps_max * n_bins), with negative values in bin 0
 *            and values at or above eps_max in bin n_bins-1 (nullable).
 * Returns 0, or -1 on bad input. */
int orc_eps_stats(const int32_t *energy, int n_groups, int group_size, const int64_t *E_gs,
                  const double *targets, int n_targets, double eps_max, int n_bins,
                  int64_t *sum, int32_t *emin, int32_t *emax, int32_t *n_le, uint32_t *hist);

/* ---- schedules and threshold tables ---------------------------------------
 * kind 0: linear  beta_s = b0 + (b1-b0) s/(S-1)
 * kind 1: geometric beta_s = b0 (b1/b0)^(s/(S-1));  S == 1 gives b0. */
int orc_schedule(int kind, double b0, double b1, int S, double *beta);
/* thr[r*K + (k-1)] = min(2^32-1, floor(exp(-2 beta_r k) 2^32)), k = 1..K.
 * A proposal with dE = 2k > 0 is accepted iff u < thr (u a Philox word). */
int orc_thresholds(const double *beta, int S, int K, uint32_t *thr);
/* Replica-exchange table for ladder pair (k, k+1):
 * thrx[k*M + (m-1)] = min(2^32-1, floor(exp(-(beta_{k+1}-beta_k) 2m) 2^32)). */
int orc_exchange_thresholds(const double *beta, int T, int M, uint32_t *thrx);

/* ---- simulated annealing ---------------------------------------------------
 * Cubic periodic lattice, L even >= 4.  Replica r (r = 0..n_rep-1) carries
 * the Philox counter word rep0 + r; chain is the fourth counter word.
 * init_random = 1 draws the initial spins from the init stream, 0 starts
 * from spins[] as given.  Sweeps sweep0 .. sweep0+S-1 use thr rows 0..S-1.
 * energy[r] = final energy; emin[r] (nullable) = lowest energy seen at the
 * end of a sweep.  check = 1 recomputes the energy after every sweep and
 * returns -2 if the tracked value differs.  Returns 0 on success. */
int orc_sa_run(int L, const int8_t *J, uint64_t seed, uint32_t chain, uint32_t rep0, int n_rep,
               const uint32_t *thr, int K, int S, int sweep0, int init_random,
               int8_t *spins, int64_t *energy, int64_t *emin, int check);

/* Same chain, with the sites of each colour visited in reverse order.  Used
 * only to show that the order inside a colour does not change the result. */
int orc_sa_run_reversed(int L, const int8_t *J, uint64_t seed, uint32_t chain, uint32_t rep0,
                        int n_rep, const uint32_t *thr, int K, int S, int sweep0,
                        int init_random, int8_t *spins, int64_t *energy);

/* ---- parallel tempering -----------------------------------------------------
 * One run = T walkers (memory slots w = 0..T-1).  pos[w] = ladder slot of
 * walker w.  Step t (t = step0 .. step0+n_steps-1): every walker makes one
 * sweep with thresholds row pos[w] and Metropolis counter (., 2t+c, w, run);
 * then ladder pairs (k, k+1) with k = t mod 2, t mod 2 + 2, ... exchange
 * walkers with probability min(1, exp(-(beta_{k+1}-beta_k) D)),
 * D = E(walker at k) - E(walker at k+1), drawn from Philox word 0 of
 * counter (k, t, 0xFFFFFFFF, run).
 * spins [T][N], energy [T], pos [T] in/out (init_random = 1 resets spins
 * from the init stream and pos to identity); emin_trace [n_steps] nullable;
 * swap_acc [T-1] nullable, accumulated. */
int orc_pt_run(int L, const int8_t *J, uint64_t seed, uint32_t run, int T,
               const uint32_t *thr, int K, const uint32_t *thrx, int M,
               int n_steps, int step0, int init_random,
               int8_t *spins, int64_t *energy, int32_t *pos,
               int64_t *emin_trace, uint32_t *swap_acc, int check);

/* ---- parallel tempering with isoenergetic cluster moves (App. D) ----------
 * The paper runs PT with isoenergetic cluster moves (ICM) and only names
 * the moves.  The move used here is Houdayer's two-replica cluster move as
 * combined with PT by Zhu, Ochoa and Katzgraber (2015), restated:
 * two copies of a T-slot ladder, walkers w = 0..2T-1, copy(w) = w / T
 * (walkers never change copy); pos[w] in [0, T) is the slot of w inside its
 * copy.  Step t:
 *   1. every walker makes one sweep with thresholds row pos[w] and
 *      Metropolis counter (., 2t+c, w, run) (as PT);
 *   2. for slots k = icm_from .. T-1: the walkers a, b of copy 0 and 1 at
 *      slot k; sites with s_a != s_b are "negative"; if there are n > 0 of
 *      them, the seed is the negative site number floor(u n / 2^32) in the
 *      order (colour, column, height) of the colour-split column layout
 *      (colour c = (x+y+z) mod 2, column x/2 + (L/2) y, height z), with u =
 *      Philox word 0 of (k, t, 0xFFFFFFFE, run); the cluster is every
 *      negative site connected to the seed through negative sites and
 *      nonzero couplings; both walkers flip the cluster (E_a + E_b is
 *      unchanged);
 *   3. in each copy cp, ladder pairs (k, k+1), k = t mod 2, t mod 2 + 2, ...
 *      exchange as in PT with u = Philox word 0 of (k + cp T, t, 0xFFFFFFFF,
 *      run) (copy 0 uses exactly PT's counters).
 * spins [2T][N], energy [2T], pos [2T] in/out (init_random resets spins from
 * the init stream with replica word w and pos[w] = w mod T); emin_trace
 * [n_steps] (minimum over all walkers after the step), swap_acc [2(T-1)]
 * (copy-major) and icm_flipped [n_steps] (sites flipped per walker by the
 * cluster moves of the step) are nullable.  check = 1 recomputes energies
 * after every phase and returns -2 on a mismatch or a change of E_a + E_b. */
int orc_pticm_run(int L, const int8_t *J, uint64_t seed, uint32_t run, int T,
                  const uint32_t *thr, int K, const uint32_t *thrx, int M,
                  int n_steps, int step0, int icm_from, int init_random,
                  int8_t *spins, int64_t *energy, int32_t *pos,
                  int64_t *emin_trace, uint32_t *swap_acc, int64_t *icm_flipped, int check);
/* One cluster move on walkers sa, sb with uniform word u (step 2 above);
 * returns the cluster size (0 when the walkers agree everywhere). */
int64_t orc_icm_move(int L, const int8_t *J, int8_t *sa, int8_t *sb, uint32_t u);

/* ---- fragment decimation (Sec. I, App. C) ----------------------------------
 * The linear-time meta-heuristic with fixed-sweep simulated annealing as the
 * subsystem optimiser.  The lattice (L even) is tiled by cores of c^3 spins
 * (L % c == 0, nb = L/c cores per axis, core k = bx + nb (by + nb bz) covers
 * [bx c, bx c + c) x ...).  The fragment of core k is the l^3 cube, l = c+2h
 * < L, that extends the core by h sites on every side (periodic).  Cores are
 * processed in phases q = 0, 1, ...; all cores of a phase see the decimation
 * state at the start of the phase.  order 0: q = (bx mod P) + P((by mod P) +
 * P (bz mod P)), P = 1 + ceil(h/c), nb % P == 0 (colour classes: no core of
 * a phase lies in another's fragment); order 1: q = bx + by + bz (a diagonal
 * wavefront: every core sees the decimated cores on its lower side).
 * Processing core k of run `run`: R independent anneals r of the fragment,
 * each as follows, with fragment site j = lx + l (ly + l lz):
 *   - site j is fixed (a boundary field) if it was decimated before the
 *     phase, else free;
 *   - bonds with both ends in the fragment count, all others are dropped;
 *   - free spins start from bit 31 of Philox word 0 of
 *     (r l^3 + j, 0xFFFFFFFF, k, run) (set: -1);
 *   - S sweeps: colour (x+y+z) mod 2 = 0 then 1, a Metropolis proposal at
 *     every free site of that colour: k_i = -s_i h_i (in-fragment bonds),
 *     flip iff k_i <= 0 or (k_i <= K and u < thr[s*K + k_i - 1]), u = Philox
 *     word 0 of (r l^3 + j, 2s + colour, k, run);
 * then the core's spins take their final values in the anneal whose
 * in-fragment energy is lowest (the smallest r among equals): they are
 * decimated.
 * dec[N] (output) holds every spin, +1/-1.  Returns 0, or -1 on bad input. */
int orc_frag_decimate(int L, const int8_t *J, int core, int halo, int R, int order, uint64_t seed,
                      uint32_t run, const uint32_t *thr, int K, int S, int8_t *dec);
/* The same with the cores of each phase visited in reverse order (the
 * result must not depend on the order inside a phase). */
int orc_frag_decimate_reversed(int L, const int8_t *J, int core, int halo, int R, int order,
                               uint64_t seed, uint32_t run, const uint32_t *thr, int K, int S,
                               int8_t *dec);
/* Anneal r of core k as above with decimation state dec (0 = not yet
 * decimated; left unchanged).  frag[l^3] receives the final fragment spins
 * (fixed ones included), *E_frag the energy of the in-fragment bonds (each
 * once). */
int orc_frag_anneal(int L, const int8_t *J, int core, int halo, int64_t k, int rep, uint64_t seed,
                    uint32_t run, const uint32_t *thr, int K, int S, const int8_t *dec,
                    int8_t *frag, int64_t *E_frag);

/* ---- initial spins (init stream) ------------------------------------------ */
void orc_init_spins(int L, uint64_t seed, uint32_t chain, uint32_t replica, int8_t *s);

/* Philox word used by the Metropolis proposal at site i, sweep s, colour c. */
uint32_t orc_metropolis_uniform(int L, uint64_t seed, uint32_t chain, uint32_t replica,
                                int s, int64_t i);

#ifdef __cplusplus
}
#endif
#endif
