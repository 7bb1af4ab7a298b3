/*
 * oracle.c -- plain C reference for the annealing hot path (test
 * infrastructure only; see oracle.h for scope and the rule that the product
 * library never loads this file).
 *
 * Written for obviousness, not speed: every Metropolis proposal recomputes
 * its local field from the six neighbours and evaluates a fresh Philox call
 * for its own random word, and the energy is always the plain sum over the
 * 3N bonds.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* lattice                                                                  */
/* ------------------------------------------------------------------------ */

static int wrap(int v, int n) { return ((v % n) + n) % n; }

int64_t orc_site(int Lx, int Ly, int Lz, int x, int y, int z)
{
    x = wrap(x, Lx);
    y = wrap(y, Ly);
    z = wrap(z, Lz);
    return (int64_t)x + (int64_t)Lx * ((int64_t)y + (int64_t)Ly * z);
}

static void coords(int Lx, int Ly, int64_t i, int *x, int *y, int *z)
{
    *x = (int)(i % Lx);
    *y = (int)((i / Lx) % Ly);
    *z = (int)(i / ((int64_t)Lx * Ly));
}

/* direction d: 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z */
static const int DX[6] = {1, -1, 0, 0, 0, 0};
static const int DY[6] = {0, 0, 1, -1, 0, 0};
static const int DZ[6] = {0, 0, 0, 0, 1, -1};

int64_t orc_nbr(int Lx, int Ly, int Lz, int64_t i, int d)
{
    int x, y, z;
    coords(Lx, Ly, i, &x, &y, &z);
    return orc_site(Lx, Ly, Lz, x + DX[d], y + DY[d], z + DZ[d]);
}

/* ------------------------------------------------------------------------ */
/* splitmix64 -- Steele, Lea, Flood, "Fast splittable pseudorandom number    */
/* generators" (OOPSLA 2014): a Weyl sequence with step 0x9E3779B97F4A7C15   */
/* followed by the 64-bit finaliser (variant 13 multipliers).               */
/* ------------------------------------------------------------------------ */

uint64_t orc_sm64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 -- Salmon, Moraes, Dror, Shaw, "Parallel random numbers:    */
/* as easy as 1, 2, 3" (SC'11).  Round: two 32x32->64 products of counter    */
/* words 0 and 2 with the multipliers, output (hi1^c1^k0, lo1, hi0^c3^k1,    */
/* lo0); the key advances by the Weyl constants between rounds.             */
/* ------------------------------------------------------------------------ */

void orc_philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* synthetic tile-planted instances (Sec. II names the tile-planting model   */
/* and its gauge scrambling; its tile classes are defined only in the        */
/* references, so the classes here are this project's own stand-ins).        */
/*                                                                          */
/* A tile is a unit cube whose lower corner has even x+y+z.  Each tile draws */
/* twelve couplings +-1 or +-2 (all nonzero), redrawn until the number of    */
/* frustrated faces equals cls.  The tile is gauged so that all-(+1) is one  */
/* of its ground states; a bond's coupling is the sum over the tiles that    */
/* contain it, so all-(+1) minimises every tile at once and E_gs is the sum */
/* of the tile minima.  A random gauge then hides the planted state.         */
/* ------------------------------------------------------------------------ */

/* corner a = ax + 2 ay + 4 az of the unit cube */
static void corner_offset(int a, int *ax, int *ay, int *az)
{
    *ax = a & 1;
    *ay = (a >> 1) & 1;
    *az = (a >> 2) & 1;
}

/* the twelve cube edges as corner pairs and their axis (0 x, 1 y, 2 z) */
static void cube_edge(int e, int *a0, int *a1, int *axis)
{
    if (e < 4) {            /* x-edges, (ay, az) = (e & 1, e >> 1) */
        int ay = e & 1, az = e >> 1;
        *a0 = 2 * ay + 4 * az;
        *a1 = *a0 + 1;
        *axis = 0;
    } else if (e < 8) {     /* y-edges, (ax, az) */
        int ax = (e - 4) & 1, az = (e - 4) >> 1;
        *a0 = ax + 4 * az;
        *a1 = *a0 + 2;
        *axis = 1;
    } else {                /* z-edges, (ax, ay) */
        int ax = (e - 8) & 1, ay = (e - 8) >> 1;
        *a0 = ax + 2 * ay;
        *a1 = *a0 + 4;
        *axis = 2;
    }
}

static int corner_coord(int a, int axis)
{
    int c[3];
    corner_offset(a, &c[0], &c[1], &c[2]);
    return c[axis];
}

/* a face (axis, side) is frustrated when the product of the signs of its
 * four edges is negative */
static int frustrated_faces(const int K[12])
{
    int axis, side, e, count = 0;
    for (axis = 0; axis < 3; ++axis) {
        for (side = 0; side < 2; ++side) {
            int negatives = 0, edges = 0;
            for (e = 0; e < 12; ++e) {
                int a0, a1, ea;
                cube_edge(e, &a0, &a1, &ea);
                if (corner_coord(a0, axis) == side && corner_coord(a1, axis) == side) {
                    ++edges;
                    if (K[e] < 0) ++negatives;
                }
            }
            if (edges != 4) abort();
            if (negatives % 2 == 1) ++count;
        }
    }
    return count;
}

static int corner_spin(int g, int a) { return ((g >> a) & 1) ? -1 : 1; }

static int tile_energy(const int K[12], int g)
{
    int e, E = 0;
    for (e = 0; e < 12; ++e) {
        int a0, a1, axis;
        cube_edge(e, &a0, &a1, &axis);
        E += K[e] * corner_spin(g, a0) * corner_spin(g, a1);
    }
    return E;
}

static void draw_tile(uint64_t seed, int64_t t, int cls, int K[12])
{
    uint64_t state = seed ^ ((uint64_t)(t + 1) * 0xD6E8FEB86659FD93ULL);
    for (;;) {
        uint64_t v = orc_sm64_next(&state);
        int e;
        for (e = 0; e < 12; ++e) {
            int negative = (int)((v >> e) & 1);
            int magnitude = ((v >> (12 + e)) & 1) ? 2 : 1;
            K[e] = negative ? -magnitude : magnitude;
        }
        if (cls < 0 || frustrated_faces(K) == cls) return;
    }
}

int orc_make_instance(int Lx, int Ly, int Lz, int periodic, int cls, uint64_t seed,
                      int8_t *J, int8_t *planted, int64_t *E_gs)
{
    int64_t N = (int64_t)Lx * Ly * Lz, i, t = 0;
    int *acc;
    int8_t *gamma;
    int x, y, z, d;
    uint64_t gstate;
    int64_t egs = 0;

    if (cls != -1 && cls != 0 && cls != 2 && cls != 4 && cls != 6) return -1;
    if (periodic) {
        if (Lx < 4 || Ly < 4 || Lz < 4 || Lx % 2 || Ly % 2 || Lz % 2) return -1;
    } else {
        if (Lx < 2 || Ly < 2 || Lz < 2) return -1;
    }
    acc = (int *)calloc((size_t)(6 * N), sizeof(int));
    gamma = (int8_t *)malloc((size_t)N);
    if (!acc || !gamma) {
        free(acc);
        free(gamma);
        return -3;
    }

    /* tiles in increasing order of their lower-corner site index */
    for (z = 0; z < (periodic ? Lz : Lz - 1); ++z)
        for (y = 0; y < (periodic ? Ly : Ly - 1); ++y)
            for (x = 0; x < (periodic ? Lx : Lx - 1); ++x) {
                int K[12], best_g = 0, best_E = 0, g, e;
                if ((x + y + z) % 2 != 0) continue;
                draw_tile(seed, t, cls, K);
                for (g = 0; g < 256; ++g) {
                    int E = tile_energy(K, g);
                    if (g == 0 || E < best_E) {
                        best_E = E;
                        best_g = g;
                    }
                }
                egs += best_E;
                for (e = 0; e < 12; ++e) {
                    int a0, a1, axis, ax0, ay0, az0, ax1, ay1, az1;
                    int kp;
                    int64_t p, q;
                    cube_edge(e, &a0, &a1, &axis);
                    kp = K[e] * corner_spin(best_g, a0) * corner_spin(best_g, a1);
                    corner_offset(a0, &ax0, &ay0, &az0);
                    corner_offset(a1, &ax1, &ay1, &az1);
                    p = orc_site(Lx, Ly, Lz, x + ax0, y + ay0, z + az0);
                    q = orc_site(Lx, Ly, Lz, x + ax1, y + ay1, z + az1);
                    /* a1 is a0 shifted by +1 along axis */
                    acc[(2 * axis) * N + p] += kp;
                    acc[(2 * axis + 1) * N + q] += kp;
                }
                ++t;
            }

    gstate = seed ^ 0xA0761D6478BD642FULL;
    for (i = 0; i < N; ++i) gamma[i] = (orc_sm64_next(&gstate) >> 63) ? -1 : 1;
    for (d = 0; d < 6; ++d)
        for (i = 0; i < N; ++i) {
            int64_t j = orc_nbr(Lx, Ly, Lz, i, d);
            int v = acc[d * N + i] * gamma[i] * gamma[j];
            if (v < -128 || v > 127) abort();
            J[d * N + i] = (int8_t)v;
        }
    for (i = 0; i < N; ++i) planted[i] = gamma[i];
    *E_gs = egs;
    free(acc);
    free(gamma);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): each nearest-neighbour pair counted once, plus sign             */
/* ------------------------------------------------------------------------ */

int64_t orc_energy(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *s)
{
    int64_t N = (int64_t)Lx * Ly * Lz, i, E = 0;
    for (i = 0; i < N; ++i) {
        int64_t sx = s[orc_nbr(Lx, Ly, Lz, i, 0)];
        int64_t sy = s[orc_nbr(Lx, Ly, Lz, i, 2)];
        int64_t sz = s[orc_nbr(Lx, Ly, Lz, i, 4)];
        E += (int64_t)s[i] * (J[0 * N + i] * sx + J[2 * N + i] * sy + J[4 * N + i] * sz);
    }
    return E;
}

int64_t orc_local_field(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *s, int64_t i)
{
    int64_t N = (int64_t)Lx * Ly * Lz, h = 0;
    int d;
    for (d = 0; d < 6; ++d) h += (int64_t)J[d * N + i] * s[orc_nbr(Lx, Ly, Lz, i, d)];
    return h;
}

/* Eq. (2) */
double orc_epsilon(int64_t E, int64_t E_gs)
{
    double gs = (double)E_gs;
    return ((double)(E - E_gs)) / fabs(gs);
}

/* The statistics App. D's TT-eps criterion reads off a set of trials: the
 * mean gap over the trials of an instance (from the exact energy sum), the
 * extremes, how many trials reach each target, and a histogram of eps. */
int orc_eps_stats(const int32_t *energy, int n_groups, int group_size, const int64_t *E_gs,
                  const double *targets, int n_targets, double eps_max, int n_bins,
                  int64_t *sum, int32_t *emin, int32_t *emax, int32_t *n_le, uint32_t *hist)
{
    int g, i, t;
    if (n_groups < 1 || group_size < 1 || n_targets < 0 || (hist && (n_bins < 1 || !(eps_max > 0.0))))
        return -1;
    for (g = 0; g < n_groups; ++g) {
        const int32_t *e = energy + (int64_t)g * group_size;
        int64_t total = 0;
        int32_t lo = e[0], hi = e[0];
        for (t = 0; t < n_targets; ++t) n_le[g * n_targets + t] = 0;
        if (hist)
            for (i = 0; i < n_bins; ++i) hist[(int64_t)g * n_bins + i] = 0;
        if (E_gs[g] == 0) return -1;
        for (i = 0; i < group_size; ++i) {
            double eps = orc_epsilon(e[i], E_gs[g]);
            total += e[i];
            if (e[i] < lo) lo = e[i];
            if (e[i] > hi) hi = e[i];
            for (t = 0; t < n_targets; ++t)
                if (eps <= targets[t]) n_le[g * n_targets + t] += 1;
            if (hist) {
                double pos = eps / eps_max * (double)n_bins;
                int b;
                if (pos < 0.0)
                    b = 0;
                else if (pos >= (double)n_bins)
                    b = n_bins - 1;
                else
                    b = (int)floor(pos);
                hist[(int64_t)g * n_bins + b] += 1;
            }
        }
        sum[g] = total;
        emin[g] = lo;
        emax[g] = hi;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* schedules and acceptance tables                                          */
/* ------------------------------------------------------------------------ */

int orc_schedule(int kind, double b0, double b1, int S, double *beta)
{
    int s;
    if (S < 1) return -1;
    if (kind == 1 && (b0 <= 0.0 || b1 <= 0.0)) return -1;
    for (s = 0; s < S; ++s) {
        double f = (S == 1) ? 0.0 : (double)s / (double)(S - 1);
        if (kind == 0)
            beta[s] = b0 + (b1 - b0) * f;
        else if (kind == 1)
            beta[s] = b0 * pow(b1 / b0, f);
        else
            return -1;
    }
    return 0;
}

static uint32_t quantise(double p)
{
    double v = ldexp(p, 32);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(v);
}

int orc_thresholds(const double *beta, int S, int K, uint32_t *thr)
{
    int s, k;
    if (S < 1 || K < 1) return -1;
    for (s = 0; s < S; ++s)
        for (k = 1; k <= K; ++k) thr[s * K + (k - 1)] = quantise(exp(-((double)(2 * k) * beta[s])));
    return 0;
}

int orc_exchange_thresholds(const double *beta, int T, int M, uint32_t *thrx)
{
    int k, m;
    if (T < 2 || M < 1) return -1;
    for (k = 0; k + 1 < T; ++k) {
        double db = beta[k + 1] - beta[k];
        for (m = 1; m <= M; ++m) thrx[k * M + (m - 1)] = quantise(exp(-((double)(2 * m) * db)));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* random streams                                                           */
/* ------------------------------------------------------------------------ */

/* init stream: site i takes word (i mod 4) of counter (i div 4, 0xFFFFFFFF,
 * replica, chain); the spin is -1 when that word's top bit is set */
void orc_init_spins(int L, uint64_t seed, uint32_t chain, uint32_t replica, int8_t *s)
{
    int64_t N = (int64_t)L * L * L, i;
    for (i = 0; i < N; ++i) {
        uint32_t ctr[4], out[4];
        ctr[0] = (uint32_t)(i / 4);
        ctr[1] = 0xFFFFFFFFu;
        ctr[2] = replica;
        ctr[3] = chain;
        orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
        s[i] = (out[i % 4] >> 31) ? -1 : 1;
    }
}

/* Metropolis stream: site (x, y, z) of colour c = (x+y+z) mod 2 lies in
 * column col = floor(x/2) + (L/2) y of its colour; the column's sites are
 * served four at a time along z, so the site takes word (z mod 4) of counter
 * (col * ceil(L/4) + floor(z/4), 2s + c, replica, chain). */
uint32_t orc_metropolis_uniform(int L, uint64_t seed, uint32_t chain, uint32_t replica,
                                int s, int64_t i)
{
    int x, y, z, c;
    int64_t col, q;
    uint32_t ctr[4], out[4];
    coords(L, L, i, &x, &y, &z);
    c = (x + y + z) % 2;
    col = (int64_t)(x / 2) + (int64_t)(L / 2) * y;
    q = col * ((L + 3) / 4) + z / 4;
    ctr[0] = (uint32_t)q;
    ctr[1] = (uint32_t)(2 * s + c);
    ctr[2] = replica;
    ctr[3] = chain;
    orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
    return out[z % 4];
}

/* ------------------------------------------------------------------------ */
/* one Metropolis proposal (App. D; acceptance min(1, exp(-beta dE)) from    */
/* the Boltzmann law of App. A).  dE = -2 s_i h_i = 2k.  k <= 0: flip.       */
/* k > 0: flip iff k <= K and u < thr_row[k-1].                             */
/* ------------------------------------------------------------------------ */

static int64_t propose(int L, const int8_t *J, int8_t *s, int64_t i, const uint32_t *thr_row,
                       int K, uint64_t seed, uint32_t chain, uint32_t replica, int sweep)
{
    int64_t h = orc_local_field(L, L, L, J, s, i);
    int64_t k = -(int64_t)s[i] * h;
    int accept;
    if (k <= 0) {
        accept = 1;
    } else {
        uint32_t u = orc_metropolis_uniform(L, seed, chain, replica, sweep, i);
        accept = (k <= K) && (u < thr_row[k - 1]);
    }
    if (!accept) return 0;
    s[i] = (int8_t)(-s[i]);
    return 2 * k;
}

/* one sweep: colour 0 then colour 1; inside a colour no two sites are
 * neighbours, so the visiting order there does not matter */
static int64_t sweep(int L, const int8_t *J, int8_t *s, const uint32_t *thr_row, int K,
                     uint64_t seed, uint32_t chain, uint32_t replica, int sw, int reversed)
{
    int64_t N = (int64_t)L * L * L, n, dE = 0;
    int c;
    for (c = 0; c < 2; ++c)
        for (n = 0; n < N; ++n) {
            int64_t i = reversed ? N - 1 - n : n;
            int x, y, z;
            coords(L, L, i, &x, &y, &z);
            if ((x + y + z) % 2 != c) continue;
            dE += propose(L, J, s, i, thr_row, K, seed, chain, replica, sw);
        }
    return dE;
}

static int sa_common(int L, const int8_t *J, uint64_t seed, uint32_t chain, uint32_t rep0,
                     int n_rep, const uint32_t *thr, int K, int S, int sweep0, int init_random,
                     int8_t *spins, int64_t *energy, int64_t *emin, int check, int reversed)
{
    int64_t N = (int64_t)L * L * L;
    int r, si;
    if (L < 4 || L % 2 || n_rep < 0 || S < 0 || K < 1 || sweep0 < 0) return -1;
    for (r = 0; r < n_rep; ++r) {
        int8_t *s = spins + (int64_t)r * N;
        uint32_t rep = rep0 + (uint32_t)r;
        int64_t E, best;
        if (init_random) orc_init_spins(L, seed, chain, rep, s);
        E = orc_energy(L, L, L, J, s);
        best = INT64_MAX;
        for (si = 0; si < S; ++si) {
            E += sweep(L, J, s, thr + (int64_t)si * K, K, seed, chain, rep, sweep0 + si, reversed);
            if (check && E != orc_energy(L, L, L, J, s)) return -2;
            if (E < best) best = E;
        }
        energy[r] = E;
        if (emin) emin[r] = (S > 0) ? best : E;
    }
    return 0;
}

int orc_sa_run(int L, const int8_t *J, uint64_t seed, uint32_t chain, uint32_t rep0, int n_rep,
               const uint32_t *thr, int K, int S, int sweep0, int init_random,
               int8_t *spins, int64_t *energy, int64_t *emin, int check)
{
    return sa_common(L, J, seed, chain, rep0, n_rep, thr, K, S, sweep0, init_random, spins,
                     energy, emin, check, 0);
}

int orc_sa_run_reversed(int L, const int8_t *J, uint64_t seed, uint32_t chain, uint32_t rep0,
                        int n_rep, const uint32_t *thr, int K, int S, int sweep0,
                        int init_random, int8_t *spins, int64_t *energy)
{
    return sa_common(L, J, seed, chain, rep0, n_rep, thr, K, S, sweep0, init_random, spins,
                     energy, NULL, 0, 1);
}

/* ------------------------------------------------------------------------ */
/* parallel tempering (App. D)                                              */
/* ------------------------------------------------------------------------ */

int orc_pt_run(int L, const int8_t *J, uint64_t seed, uint32_t run, int T,
               const uint32_t *thr, int K, const uint32_t *thrx, int M,
               int n_steps, int step0, int init_random,
               int8_t *spins, int64_t *energy, int32_t *pos,
               int64_t *emin_trace, uint32_t *swap_acc, int check)
{
    int64_t N = (int64_t)L * L * L;
    int w, k, ti;
    int32_t *who;
    if (L < 4 || L % 2 || T < 2 || K < 1 || M < 1 || n_steps < 0 || step0 < 0) return -1;
    who = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    if (!who) return -3;
    if (init_random)
        for (w = 0; w < T; ++w) {
            orc_init_spins(L, seed, run, (uint32_t)w, spins + (int64_t)w * N);
            pos[w] = w;
        }
    for (k = 0; k < T; ++k) who[k] = -1;
    for (w = 0; w < T; ++w) {
        if (pos[w] < 0 || pos[w] >= T || who[pos[w]] != -1) {
            free(who);
            return -1;
        }
        who[pos[w]] = w;
        energy[w] = orc_energy(L, L, L, J, spins + (int64_t)w * N);
    }
    for (ti = 0; ti < n_steps; ++ti) {
        int t = step0 + ti;
        int64_t best;
        for (w = 0; w < T; ++w) {
            int8_t *s = spins + (int64_t)w * N;
            energy[w] += sweep(L, J, s, thr + (int64_t)pos[w] * K, K, seed, run, (uint32_t)w, t, 0);
            if (check && energy[w] != orc_energy(L, L, L, J, s)) {
                free(who);
                return -2;
            }
        }
        for (k = t % 2; k + 1 < T; k += 2) {
            int a = who[k], b = who[k + 1];
            int64_t D = energy[a] - energy[b];
            int accept;
            if (D <= 0) {
                accept = 1;
            } else {
                uint32_t ctr[4], out[4];
                int64_t m = D / 2;
                ctr[0] = (uint32_t)k;
                ctr[1] = (uint32_t)t;
                ctr[2] = 0xFFFFFFFFu;
                ctr[3] = run;
                orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
                accept = (m <= M) && (out[0] < thrx[(int64_t)k * M + (m - 1)]);
            }
            if (accept) {
                who[k] = b;
                who[k + 1] = a;
                pos[b] = k;
                pos[a] = k + 1;
                if (swap_acc) swap_acc[k] += 1;
            }
        }
        best = energy[0];
        for (w = 1; w < T; ++w)
            if (energy[w] < best) best = energy[w];
        if (emin_trace) emin_trace[ti] = best;
    }
    free(who);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* fragment decimation (Sec. I: bootstrapped subsystem optimisation with a   */
/* fixed-time stochastic optimiser; App. C: fragments overlapping earlier    */
/* decimations, non-overlapping fragments processed together)               */
/* ------------------------------------------------------------------------ */

/* the colour-class order needs nb % P == 0 so that cores of one class stay
 * P cores apart across the periodic wrap; the wavefront order needs nothing */
static int frag_params_ok(int L, int c, int h, int order)
{
    int l = c + 2 * h, nb, P;
    if (L < 4 || L % 2 || c < 1 || h < 0 || L % c || l >= L) return 0;
    nb = L / c;
    P = 1 + (h + c - 1) / c;
    return order != 0 || nb % P == 0;
}

static uint32_t frag_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int w)
{
    uint32_t ctr[4], out[4];
    ctr[0] = c0;
    ctr[1] = c1;
    ctr[2] = c2;
    ctr[3] = c3;
    orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
    return out[w];
}

int orc_frag_anneal(int L, const int8_t *J, int core, int halo, int64_t k, int rep, uint64_t seed,
                    uint32_t run, const uint32_t *thr, int K, int S, const int8_t *dec,
                    int8_t *frag, int64_t *E_frag)
{
    int l = core + 2 * halo, nb, bx, by, bz, lx, ly, lz, d, s, col;
    int64_t N = (int64_t)L * L * L, n3, j, E;
    int64_t *g;
    int8_t *fixed;
    uint32_t w0;
    if (!frag_params_ok(L, core, halo, 1) || K < 1 || S < 0 || rep < 0) return -1;
    nb = L / core;
    if (k < 0 || k >= (int64_t)nb * nb * nb) return -1;
    bx = (int)(k % nb);
    by = (int)((k / nb) % nb);
    bz = (int)(k / ((int64_t)nb * nb));
    n3 = (int64_t)l * l * l;
    w0 = (uint32_t)rep * (uint32_t)n3;   /* counter word 0 = rep l^3 + j */
    g = (int64_t *)malloc(sizeof(int64_t) * (size_t)n3);
    fixed = (int8_t *)malloc((size_t)n3);
    if (!g || !fixed) return -3;
    /* fragment sites, their global index and state */
    for (lz = 0; lz < l; ++lz)
        for (ly = 0; ly < l; ++ly)
            for (lx = 0; lx < l; ++lx) {
                j = lx + (int64_t)l * (ly + (int64_t)l * lz);
                g[j] = orc_site(L, L, L, wrap(bx * core - halo + lx, L), wrap(by * core - halo + ly, L),
                                wrap(bz * core - halo + lz, L));
                fixed[j] = dec[g[j]] != 0;
                if (fixed[j])
                    frag[j] = dec[g[j]];
                else
                    frag[j] = (frag_word(seed, w0 + (uint32_t)j, 0xFFFFFFFFu, (uint32_t)k, run, 0) >> 31) ? -1 : 1;
            }
    /* sweeps over the free sites, colour by colour */
    for (s = 0; s < S; ++s)
        for (col = 0; col < 2; ++col)
            for (j = 0; j < n3; ++j) {
                int x, y, z;
                int64_t hfield = 0, kk;
                int acc;
                if (fixed[j]) continue;
                coords(L, L, g[j], &x, &y, &z);
                if ((x + y + z) % 2 != col) continue;
                lx = (int)(j % l);
                ly = (int)((j / l) % l);
                lz = (int)(j / ((int64_t)l * l));
                for (d = 0; d < 6; ++d) {
                    int mx = lx + (d == 0) - (d == 1), my = ly + (d == 2) - (d == 3), mz = lz + (d == 4) - (d == 5);
                    if (mx < 0 || mx >= l || my < 0 || my >= l || mz < 0 || mz >= l) continue; /* bond leaves */
                    hfield += (int64_t)J[(int64_t)d * N + g[j]] * frag[mx + (int64_t)l * (my + (int64_t)l * mz)];
                }
                kk = -(int64_t)frag[j] * hfield;
                if (kk <= 0)
                    acc = 1;
                else
                    /* sweeps 4m..4m+3 of a site use words 0..3 of one call */
                    acc = kk <= K && frag_word(seed, w0 + (uint32_t)j, (uint32_t)(2 * (s / 4) + col), (uint32_t)k, run,
                                               s % 4) < thr[(int64_t)s * K + (kk - 1)];
                if (acc) frag[j] = (int8_t)(-frag[j]);
            }
    /* energy of the in-fragment bonds (+x, +y, +z partners inside) */
    E = 0;
    for (j = 0; j < n3; ++j) {
        lx = (int)(j % l);
        ly = (int)((j / l) % l);
        lz = (int)(j / ((int64_t)l * l));
        if (lx + 1 < l) E += (int64_t)J[0 * N + g[j]] * frag[j] * frag[j + 1];
        if (ly + 1 < l) E += (int64_t)J[2 * N + g[j]] * frag[j] * frag[j + l];
        if (lz + 1 < l) E += (int64_t)J[4 * N + g[j]] * frag[j] * frag[j + (int64_t)l * l];
    }
    *E_frag = E;
    free(g);
    free(fixed);
    return 0;
}

/* phase of core (bx, by, bz): order 0 = colour classes
 * (bx mod P) + P((by mod P) + P(bz mod P)); order 1 = diagonal wavefront
 * bx + by + bz */
static int frag_phase(int order, int P, int bx, int by, int bz)
{
    return order == 0 ? (bx % P) + P * ((by % P) + P * (bz % P)) : bx + by + bz;
}

static int frag_common(int L, const int8_t *J, int core, int halo, int R, int order, uint64_t seed,
                       uint32_t run, const uint32_t *thr, int K, int S, int8_t *dec, int reversed)
{
    int l = core + 2 * halo, nb, P, q, r, nq;
    int64_t N = (int64_t)L * L * L, ncores, n, i;
    int8_t *frag, *best, *snap;
    if (order < 0 || order > 1 || !frag_params_ok(L, core, halo, order) || K < 1 || S < 0 || R < 1) return -1;
    nb = L / core;
    P = 1 + (halo + core - 1) / core;
    nq = order == 0 ? P * P * P : 3 * (nb - 1) + 1;
    ncores = (int64_t)nb * nb * nb;
    frag = (int8_t *)malloc((size_t)l * l * l);
    best = (int8_t *)malloc((size_t)l * l * l);
    snap = (int8_t *)malloc((size_t)N);
    if (!frag || !best || !snap) return -3;
    for (i = 0; i < N; ++i) dec[i] = 0;
    for (q = 0; q < nq; ++q) {
        /* every core of a phase sees the decimation state at the start of
         * the phase */
        memcpy(snap, dec, (size_t)N);
        for (n = 0; n < ncores; ++n) {
            int64_t k = reversed ? ncores - 1 - n : n, E, Ebest = INT64_MAX;
            int bx = (int)(k % nb), by = (int)((k / nb) % nb), bz = (int)(k / ((int64_t)nb * nb));
            int cx, cy, cz;
            if (frag_phase(order, P, bx, by, bz) != q) continue;
            /* R independent anneals of the fragment; the lowest fragment
             * energy wins (the first replica among equals) */
            for (r = 0; r < R; ++r) {
                if (orc_frag_anneal(L, J, core, halo, k, r, seed, run, thr, K, S, snap, frag, &E)) {
                    free(frag);
                    free(best);
                    free(snap);
                    return -1;
                }
                if (E < Ebest) {
                    Ebest = E;
                    memcpy(best, frag, (size_t)l * l * l);
                }
            }
            /* the core sits at offset halo inside the fragment */
            for (cz = 0; cz < core; ++cz)
                for (cy = 0; cy < core; ++cy)
                    for (cx = 0; cx < core; ++cx) {
                        int64_t j = (halo + cx) + (int64_t)l * ((halo + cy) + (int64_t)l * (halo + cz));
                        dec[orc_site(L, L, L, bx * core + cx, by * core + cy, bz * core + cz)] = best[j];
                    }
        }
    }
    free(frag);
    free(best);
    free(snap);
    return 0;
}

int orc_frag_decimate(int L, const int8_t *J, int core, int halo, int R, int order, uint64_t seed,
                      uint32_t run, const uint32_t *thr, int K, int S, int8_t *dec)
{
    return frag_common(L, J, core, halo, R, order, seed, run, thr, K, S, dec, 0);
}

int orc_frag_decimate_reversed(int L, const int8_t *J, int core, int halo, int R, int order,
                               uint64_t seed, uint32_t run, const uint32_t *thr, int K, int S,
                               int8_t *dec)
{
    return frag_common(L, J, core, halo, R, order, seed, run, thr, K, S, dec, 1);
}

/* ------------------------------------------------------------------------ */
/* parallel tempering with isoenergetic cluster moves (App. D)              */
/* ------------------------------------------------------------------------ */

int64_t orc_icm_move(int L, const int8_t *J, int8_t *sa, int8_t *sb, uint32_t u)
{
    int64_t N = (int64_t)L * L * L, n = 0, idx, seed_site = -1, head, tail, i;
    int64_t *queue;
    int8_t *in;
    int c, col, z, d, H = L / 2;
    /* negative sites in the order (colour, column, height) */
    for (c = 0; c < 2; ++c)
        for (col = 0; col < H * L; ++col)
            for (z = 0; z < L; ++z) {
                int y = col / H, x = 2 * (col % H) + ((y + z + c) & 1);
                i = orc_site(L, L, L, x, y, z);
                if (sa[i] != sb[i]) ++n;
            }
    if (n == 0) return 0;
    idx = (int64_t)(((uint64_t)u * (uint64_t)n) >> 32);
    for (c = 0; c < 2 && seed_site < 0; ++c)
        for (col = 0; col < H * L && seed_site < 0; ++col)
            for (z = 0; z < L; ++z) {
                int y = col / H, x = 2 * (col % H) + ((y + z + c) & 1);
                i = orc_site(L, L, L, x, y, z);
                if (sa[i] != sb[i] && idx-- == 0) {
                    seed_site = i;
                    break;
                }
            }
    /* breadth-first growth through negative sites and nonzero couplings */
    queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    in = (int8_t *)calloc((size_t)N, 1);
    if (!queue || !in) return -3;
    head = tail = 0;
    queue[tail++] = seed_site;
    in[seed_site] = 1;
    while (head < tail) {
        i = queue[head++];
        for (d = 0; d < 6; ++d) {
            int64_t j = orc_nbr(L, L, L, i, d);
            if (J[(int64_t)d * N + i] == 0 || in[j] || sa[j] == sb[j]) continue;
            in[j] = 1;
            queue[tail++] = j;
        }
    }
    for (head = 0; head < tail; ++head) {
        i = queue[head];
        sa[i] = (int8_t)(-sa[i]);
        sb[i] = (int8_t)(-sb[i]);
    }
    free(queue);
    free(in);
    return tail;
}

int orc_pticm_run(int L, const int8_t *J, uint64_t seed, uint32_t run, int T,
                  const uint32_t *thr, int K, const uint32_t *thrx, int M,
                  int n_steps, int step0, int icm_from, int init_random,
                  int8_t *spins, int64_t *energy, int32_t *pos,
                  int64_t *emin_trace, uint32_t *swap_acc, int64_t *icm_flipped, int check)
{
    int64_t N = (int64_t)L * L * L;
    int w, k, ti, cp, W = 2 * T;
    int32_t *who;   /* who[cp*T + k] = walker of copy cp at slot k */
    if (L < 4 || L % 2 || T < 2 || K < 1 || M < 1 || n_steps < 0 || step0 < 0 || icm_from < 0) return -1;
    who = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    if (!who) return -3;
    if (init_random)
        for (w = 0; w < W; ++w) {
            orc_init_spins(L, seed, run, (uint32_t)w, spins + (int64_t)w * N);
            pos[w] = w % T;
        }
    for (k = 0; k < W; ++k) who[k] = -1;
    for (w = 0; w < W; ++w) {
        int slot = (w / T) * T + pos[w];
        if (pos[w] < 0 || pos[w] >= T || who[slot] != -1) {
            free(who);
            return -1;
        }
        who[slot] = w;
        energy[w] = orc_energy(L, L, L, J, spins + (int64_t)w * N);
    }
    for (ti = 0; ti < n_steps; ++ti) {
        int t = step0 + ti;
        int64_t best, flipped = 0;
        /* 1. sweeps */
        for (w = 0; w < W; ++w) {
            int8_t *s = spins + (int64_t)w * N;
            energy[w] += sweep(L, J, s, thr + (int64_t)pos[w] * K, K, seed, run, (uint32_t)w, t, 0);
            if (check && energy[w] != orc_energy(L, L, L, J, s)) {
                free(who);
                return -2;
            }
        }
        /* 2. cluster moves between the copies, slot by slot */
        for (k = icm_from; k < T; ++k) {
            int a = who[k], b = who[T + k];
            int64_t before = energy[a] + energy[b], size;
            uint32_t ctr[4], out[4];
            ctr[0] = (uint32_t)k;
            ctr[1] = (uint32_t)t;
            ctr[2] = 0xFFFFFFFEu;
            ctr[3] = run;
            orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
            size = orc_icm_move(L, J, spins + (int64_t)a * N, spins + (int64_t)b * N, out[0]);
            if (size < 0) {
                free(who);
                return -3;
            }
            flipped += size;
            energy[a] = orc_energy(L, L, L, J, spins + (int64_t)a * N);
            energy[b] = orc_energy(L, L, L, J, spins + (int64_t)b * N);
            if (check && energy[a] + energy[b] != before) {
                free(who);
                return -2;
            }
        }
        /* 3. exchanges inside each copy */
        for (cp = 0; cp < 2; ++cp)
            for (k = t % 2; k + 1 < T; k += 2) {
                int a = who[cp * T + k], b = who[cp * T + k + 1];
                int64_t D = energy[a] - energy[b];
                int accept;
                if (D <= 0) {
                    accept = 1;
                } else {
                    uint32_t ctr[4], out[4];
                    int64_t m = D / 2;
                    ctr[0] = (uint32_t)(k + cp * T);
                    ctr[1] = (uint32_t)t;
                    ctr[2] = 0xFFFFFFFFu;
                    ctr[3] = run;
                    orc_philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
                    accept = (m <= M) && (out[0] < thrx[(int64_t)k * M + (m - 1)]);
                }
                if (accept) {
                    who[cp * T + k] = b;
                    who[cp * T + k + 1] = a;
                    pos[b] = k;
                    pos[a] = k + 1;
                    if (swap_acc) swap_acc[cp * (T - 1) + k] += 1;
                }
            }
        best = energy[0];
        for (w = 1; w < W; ++w)
            if (energy[w] < best) best = energy[w];
        if (emin_trace) emin_trace[ti] = best;
        if (icm_flipped) icm_flipped[ti] = flipped;
    }
    free(who);
    return 0;
}
