/*
 * bruteforce.c -- test helper, independent of the oracle: exhaustive
 * enumeration of every spin configuration of a tiny system given as an
 * explicit bond list (i, j, J_ij), energy sum over bonds of J_ij s_i s_j
 * (Eq. 1 of the paper).  Configurations are visited in Gray-code order so
 * that each step flips one spin and updates the energy by that spin's
 * local field.  Writes the minimum energy and the number of states at each
 * energy (density of states g(E) for E in [emin_bound, emin_bound+nbins)).
 */
#include <stdint.h>
#include <stdlib.h>

int bf_enumerate(int n_spins, int n_bonds, const int32_t *bi, const int32_t *bj,
                 const int32_t *bJ, int64_t emin_bound, int64_t nbins,
                 int64_t *min_energy, uint64_t *dos)
{
    int8_t *s;
    int64_t *field;   /* field[i] = sum_j J_ij s_j over bonds touching i */
    int32_t *deg, *adj, *adjJ;   /* adjacency lists, at most 64 per spin */
    int64_t E = 0, best;
    uint64_t n, total;
    int b;
    if (n_spins < 1 || n_spins > 40) return -1;
    s = (int8_t *)malloc((size_t)n_spins);
    field = (int64_t *)calloc((size_t)n_spins, sizeof(int64_t));
    deg = (int32_t *)calloc((size_t)n_spins, sizeof(int32_t));
    adj = (int32_t *)malloc(sizeof(int32_t) * 64 * (size_t)n_spins);
    adjJ = (int32_t *)malloc(sizeof(int32_t) * 64 * (size_t)n_spins);
    if (!s || !field || !deg || !adj || !adjJ) return -3;
    for (b = 0; b < n_bonds; ++b) {
        if (deg[bi[b]] >= 64 || deg[bj[b]] >= 64) return -1;
        adj[64 * bi[b] + deg[bi[b]]] = bj[b];
        adjJ[64 * bi[b] + deg[bi[b]]++] = bJ[b];
        adj[64 * bj[b] + deg[bj[b]]] = bi[b];
        adjJ[64 * bj[b] + deg[bj[b]]++] = bJ[b];
    }
    for (b = 0; b < n_spins; ++b) s[b] = 1;
    for (b = 0; b < n_bonds; ++b) {
        E += (int64_t)bJ[b];
        field[bi[b]] += bJ[b];
        field[bj[b]] += bJ[b];
    }
    best = E;
    total = (uint64_t)1 << n_spins;
    if (dos) {
        int64_t k = E - emin_bound;
        if (k < 0 || k >= nbins) return -2;
        dos[k] += 1;
    }
    for (n = 1; n < total; ++n) {
        int flip = __builtin_ctzll(n);
        int8_t old = s[flip];
        E += -2 * (int64_t)old * field[flip];
        s[flip] = (int8_t)(-old);
        for (b = 0; b < deg[flip]; ++b)
            field[adj[64 * flip + b]] += -2 * (int64_t)old * adjJ[64 * flip + b];
        if (E < best) best = E;
        if (dos) {
            int64_t k = E - emin_bound;
            if (k < 0 || k >= nbins) return -2;
            dos[k] += 1;
        }
    }
    *min_energy = best;
    free(s);
    free(field);
    free(deg);
    free(adj);
    free(adjJ);
    return 0;
}
