// tn_plan.cpp -- host planner of the tensor-network fragment decimation
// (Sec. I, App. A-C): the distinct fragment shapes of a phase order, an
// elimination program for each, and the per-phase work lists.
//
// The free set of a fragment depends only on the phases of its sites
// relative to the centre's, so a lattice has few distinct shapes (at most a
// few hundred at l = 5).  For each shape the planner tries the 48 sweeps
// that eliminate spins in lexicographic order of a signed permutation of
// the coordinates, 48 that sweep diagonal planes, and a greedy order that
// always eliminates the spin adding the fewest new active spins, and keeps
// the one with the smallest table (then the least work).
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <new>
#include <stdexcept>
#include <numeric>

#include "common.hpp"
#include "tn.hpp"

namespace sg {

int tn_phase_of(int order, int L, int h, int x, int y, int z)
{
    (void)L;
    const int P = 1 + h;
    return order == 0 ? (x % P) + P * ((y % P) + P * (z % P)) : x + y + z;
}

int tn_n_phases(int order, int L, int h)
{
    const int P = 1 + h;
    return order == 0 ? P * P * P : 3 * (L - 1) + 1;
}

namespace {

using Mask = std::array<uint64_t, 2>;   // bit j: local site j is free (l^3 <= 125)

inline bool bit(const Mask &m, int j) { return (m[j >> 6] >> (j & 63)) & 1u; }

struct Frag {
    int l, n3, c;
    Mask free;
    int nbr(int j, int d) const
    {
        int x = j % l, y = (j / l) % l, z = j / (l * l);
        x += (d == 0) - (d == 1);
        y += (d == 2) - (d == 3);
        z += (d == 4) - (d == 5);
        if (x < 0 || y < 0 || z < 0 || x >= l || y >= l || z >= l) return -1;
        return x + l * (y + l * z);
    }
    bool is_free(int j) const { return j != c && bit(free, j); }
};

struct Cost {
    int W = 0;
    double work = 0;   // sum over steps of 2^(active spins)
};

// table size and work of eliminating in `order`
Cost evaluate(const Frag &f, const std::vector<int> &order)
{
    std::vector<char> act(f.n3, 0), done(f.n3, 0);
    int n_act = 0;
    Cost c;
    for (int v : order) {
        if (!act[v]) act[v] = 1, ++n_act;
        for (int d = 0; d < 6; ++d) {
            const int u = f.nbr(v, d);
            if (u >= 0 && f.is_free(u) && !done[u] && !act[u]) act[u] = 1, ++n_act;
        }
        c.W = std::max(c.W, n_act);
        c.work += static_cast<double>(int64_t{1} << std::min(n_act, 62));
        act[v] = 0, --n_act;
        done[v] = 1;
    }
    return c;
}

std::vector<int> greedy_order(const Frag &f, const std::vector<int> &V)
{
    std::vector<char> act(f.n3, 0), done(f.n3, 0);
    std::vector<int> order, rest = V;
    int n_act = 0;
    while (!rest.empty()) {
        int best = -1, bk0 = 0, bk1 = 0;
        for (size_t i = 0; i < rest.size(); ++i) {
            const int v = rest[i];
            int add = act[v] ? 0 : 1, linked = 0;
            for (int d = 0; d < 6; ++d) {
                const int u = f.nbr(v, d);
                if (u >= 0 && f.is_free(u) && !done[u]) {
                    if (act[u])
                        ++linked;
                    else
                        ++add;
                }
            }
            const int k0 = n_act + add, k1 = -linked;
            if (best < 0 || k0 < bk0 || (k0 == bk0 && k1 < bk1)) best = static_cast<int>(i), bk0 = k0, bk1 = k1;
        }
        const int v = rest[best];
        rest.erase(rest.begin() + best);
        if (!act[v]) act[v] = 1, ++n_act;
        for (int d = 0; d < 6; ++d) {
            const int u = f.nbr(v, d);
            if (u >= 0 && f.is_free(u) && !done[u] && !act[u]) act[u] = 1, ++n_act;
        }
        act[v] = 0, --n_act;
        done[v] = 1;
        order.push_back(v);
    }
    return order;
}

std::vector<int> best_order(const Frag &f, const std::vector<int> &V)
{
    std::vector<std::vector<int>> cands;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    auto coord = [&](int j, int a) { return a == 0 ? j % f.l : a == 1 ? (j / f.l) % f.l : j / (f.l * f.l); };
    for (int diag = 0; diag < 2; ++diag)
        for (const auto &p : perms)
            for (int sg = 0; sg < 8; ++sg) {
                const int s[3] = {(sg & 1) ? -1 : 1, (sg & 2) ? -1 : 1, (sg & 4) ? -1 : 1};
                auto key = [&](int j) {
                    std::array<int, 4> k{};
                    k[0] = diag ? s[0] * coord(j, 0) + s[1] * coord(j, 1) + s[2] * coord(j, 2) : 0;
                    for (int a = 0; a < 3; ++a) k[1 + a] = (diag ? 1 : s[a]) * coord(j, p[a]);
                    return k;
                };
                std::vector<int> o = V;
                std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return key(a) < key(b); });
                cands.push_back(std::move(o));
            }
    cands.push_back(greedy_order(f, V));
    size_t bi = 0;
    Cost bc = evaluate(f, cands[0]);
    for (size_t i = 1; i < cands.size(); ++i) {
        const Cost c = evaluate(f, cands[i]);
        if (c.W < bc.W || (c.W == bc.W && c.work < bc.work)) bi = i, bc = c;
    }
    return cands[bi];
}

// the elimination program of one shape
// the shape's rounds (see TnRound), pairing its steps greedily from the first
void plan_rounds(TnShape &sh, const std::vector<TnStep> &steps, std::vector<TnRound> &rounds)
{
    sh.round0 = static_cast<int32_t>(rounds.size());
    for (int t = 0; t < sh.n_steps;) {
        const TnStep &s0 = steps[sh.step0 + t];
        TnRound R{};
        R.step = static_cast<int16_t>(t);
        R.read_bits = s0.n_base;
        if (t + 2 < sh.n_steps) {
            const TnStep &s1 = steps[sh.step0 + t + 1];
            uint32_t base = 0;
            for (int r = 0; r < s0.n_runs; ++r) base |= ((1u << s0.run_len[r]) - 1u) << s0.run_start[r];
            const uint32_t bbit = 1u << s1.a;
            const int mode = (base & bbit) ? 1 : (s0.newmask & bbit) ? 2 : 0;
            const int kept = (1 << __builtin_popcount(s0.newmask)) * (mode == 1 ? 2 : 1);
            if (kept <= kTnFuseMax && s1.a_active == (mode != 0) && s1.a != s0.a) {
                R.fused = 1;
                R.b_mode = static_cast<uint8_t>(mode);
                if (mode == 1) {
                    R.b_rank = static_cast<uint8_t>(__builtin_popcount(base & (bbit - 1u)));
                    R.read_bits = static_cast<uint8_t>(s0.n_base - 1);
                }
            }
        }
        rounds.push_back(R);
        t += 1 + R.fused;
    }
    sh.n_rounds = static_cast<int32_t>(rounds.size()) - sh.round0;
}

TnShape plan_shape(const Frag &f, std::vector<TnStep> &steps)
{
    std::vector<int> V;
    for (int j = 0; j < f.n3; ++j)
        if (f.is_free(j)) V.push_back(j);
    const std::vector<int> order = best_order(f, V);
    TnShape sh{};
    sh.step0 = static_cast<int32_t>(steps.size());
    sh.n_steps = static_cast<int32_t>(order.size());
    for (int d = 0; d < 6; ++d) {
        const int u = f.nbr(f.c, d);
        sh.ccode[d] = (u >= 0 && !bit(f.free, u)) ? kTnConst : kTnNone;
    }
    // elimination position of every free spin, and the least table width:
    // the most spins active at once (lowest-free assignment)
    std::vector<int> pos(f.n3, -1);
    for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = static_cast<int>(i);
    int wmin = 0;
    {
        std::vector<char> act(f.n3, 0), dn(f.n3, 0);
        int n_act = 0;
        for (int v : order) {
            if (!act[v]) act[v] = 1, ++n_act;
            for (int d = 0; d < 6; ++d) {
                const int u = f.nbr(v, d);
                if (u >= 0 && u != f.c && f.is_free(u) && !dn[u] && !act[u]) act[u] = 1, ++n_act;
            }
            wmin = std::max(wmin, n_act);
            dn[v] = 1;
            --n_act;
        }
    }
    std::vector<int> slot(f.n3, -1);
    std::vector<char> done(f.n3, 0);
    uint64_t used = 0;   // slot occupancy
    // a spin's slot: counted from the bottom, as many slots as active spins
    // that outlive it (so long-lived spins sit on the low bits), the nearest
    // free one at or above that, else below; never at or above wmin
    auto take_for = [&](int w) {
        int later = 0;
        for (int u = 0; u < f.n3; ++u)
            if (slot[u] >= 0 && !done[u] && pos[u] > pos[w]) ++later;
        later = std::min(later, wmin - 1);
        int s = -1;
        for (int q = later; q < wmin && s < 0; ++q)
            if (!((used >> q) & 1u)) s = q;
        for (int q = later - 1; q >= 0 && s < 0; --q)
            if (!((used >> q) & 1u)) s = q;
        // never: at most wmin spins are active at once
        if (s < 0) throw std::length_error("no free slot below the least table width");
        used |= uint64_t{1} << s;
        return s;
    };
    int W = 0, max_base = 0;
    uint64_t P = 0;   // canonical (active) slots before the step
    for (int v : order) {
        if (slot[v] < 0) slot[v] = take_for(v);
        TnStep st{};
        st.lv = static_cast<int16_t>(v);
        for (int d = 0; d < 6; ++d) {
            const int u = f.nbr(v, d);
            int8_t code;
            if (u < 0 || (f.is_free(u) && done[u]))
                code = kTnNone;
            else if (u == f.c)
                code = kTnCentre;
            else if (!f.is_free(u))
                code = kTnConst;
            else {
                if (slot[u] < 0) slot[u] = take_for(u);
                code = static_cast<int8_t>(slot[u]);
            }
            st.code[d] = code;
        }
        st.a = static_cast<uint8_t>(slot[v]);
        for (int s = 63; s >= 0; --s)
            if ((used >> s) & 1u) {
                W = std::max(W, s + 1);
                break;
            }
        // canonical bookkeeping of the workspace tier: the slots active now
        // are exactly `used`; those not in P are new at this step
        const uint64_t abit = uint64_t{1} << st.a;
        const uint64_t fresh = used & ~P;
        const uint64_t base = P & ~abit;
        st.a_active = (P & abit) ? 1 : 0;
        st.newmask = static_cast<uint32_t>(fresh & ~abit);
        int n_runs = 0, n_base = 0;
        for (int b = 0; b < 64;) {
            if (!((base >> b) & 1u)) {
                ++b;
                continue;
            }
            int e = b;
            while (e < 64 && ((base >> e) & 1u)) ++e;
            if (n_runs == 8) throw std::length_error("an elimination step needs more than 8 slot runs");
            st.run_start[n_runs] = static_cast<uint8_t>(b);
            st.run_len[n_runs] = static_cast<uint8_t>(e - b);
            ++n_runs;
            n_base += e - b;
            b = e;
        }
        st.n_runs = static_cast<uint8_t>(n_runs);
        st.n_base = static_cast<uint8_t>(n_base);
        max_base = std::max(max_base, n_base);
        used &= ~(uint64_t{1} << slot[v]);
        P = used;
        done[v] = 1;
        steps.push_back(st);
    }
    sh.W = W;
    sh.max_base = static_cast<int16_t>(max_base);
    return sh;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int sg_tn_plan_create(int32_t L, int32_t halo, int32_t order, int32_t lds_max_bits, sg_tn_plan **out)
{
    if (!out) return fail(SG_EINVAL, "sg_tn_plan_create: out is NULL");
    *out = nullptr;
    if (!lattice_ok(L)) return fail(SG_EINVAL, "sg_tn_plan_create: L = %d", L);
    if (halo < 0 || halo > SG_TN_MAX_HALO || 2 * halo + 1 >= L)
        return fail(SG_EINVAL, "sg_tn_plan_create: halo = %d (l = 2h + 1 must be < L, h <= %d)", halo,
                    SG_TN_MAX_HALO);
    if (order != 0 && order != 1) return fail(SG_EINVAL, "sg_tn_plan_create: order = %d", order);
    if (order == 0 && L % (1 + halo) != 0)
        return fail(SG_EINVAL, "sg_tn_plan_create: colour classes need L %% (1 + h) == 0 (L = %d, h = %d)", L, halo);
    if (lds_max_bits == 0) lds_max_bits = SG_TN_LDS_BITS;
    if (lds_max_bits < 1 || lds_max_bits > SG_TN_LDS_BITS)
        return fail(SG_EINVAL, "sg_tn_plan_create: lds_max_bits = %d", lds_max_bits);
    clear_error();

    sg_tn_plan *p = new (std::nothrow) sg_tn_plan;
    if (!p) return fail(SG_ENOMEM, "sg_tn_plan_create: host allocation");
    try {
        p->L = L;
        p->h = halo;
        p->l = 2 * halo + 1;
        p->order = order;
        p->lds_bits = lds_max_bits;
        const int l = p->l, n3 = l * l * l;
        const int nq = tn_n_phases(order, L, halo);
        const int64_t N = static_cast<int64_t>(L) * L * L;
        std::vector<int> ph(N);
        for (int64_t i = 0; i < N; ++i)
            ph[i] = tn_phase_of(order, L, halo, static_cast<int>(i % L), static_cast<int>((i / L) % L),
                                static_cast<int>(i / (static_cast<int64_t>(L) * L)));
        std::map<Mask, int> ids;
        std::vector<std::vector<TnItem>> by_phase(nq);
        for (int64_t i = 0; i < N; ++i) {
            const int x0 = static_cast<int>(i % L), y0 = static_cast<int>((i / L) % L),
                      z0 = static_cast<int>(i / (static_cast<int64_t>(L) * L));
            Mask m{0, 0};
            for (int j = 0; j < n3; ++j) {
                const int gx = (x0 + j % l - halo + L) % L, gy = (y0 + (j / l) % l - halo + L) % L,
                          gz = (z0 + j / (l * l) - halo + L) % L;
                if (ph[gx + static_cast<int64_t>(L) * (gy + static_cast<int64_t>(L) * gz)] >= ph[i])
                    m[j >> 6] |= uint64_t{1} << (j & 63);
            }
            auto it = ids.find(m);
            int id;
            if (it == ids.end()) {
                Frag f{l, n3, n3 / 2, m};
                TnShape sh = plan_shape(f, p->steps);
                plan_rounds(sh, p->steps, p->rounds);
                if (sh.W > SG_TN_MAX_BITS) {
                    delete p;
                    return fail(SG_EUNSUPPORTED, "sg_tn_plan_create: a fragment needs a table of 2^%d entries", sh.W);
                }
                id = static_cast<int>(p->shapes.size());
                p->shapes.push_back(sh);
                ids.emplace(m, id);
            } else {
                id = it->second;
            }
            by_phase[ph[i]].push_back(TnItem{static_cast<int32_t>(i), id});
        }
        p->phases.resize(nq);
        for (int q = 0; q < nq; ++q) {
            TnPhase &P = p->phases[q];
            P = TnPhase{};
            P.item0 = static_cast<int32_t>(p->items.size());
            std::vector<TnItem> hbm;
            for (const TnItem &it : by_phase[q]) {
                const TnShape &sh = p->shapes[it.shape];
                p->max_bits = std::max(p->max_bits, sh.W);
                p->max_steps = std::max(p->max_steps, sh.n_steps);
                p->pair_updates += 2.0 * sh.n_steps * static_cast<double>(sh.W > 0 ? int64_t{1} << (sh.W - 1) : 0);
                if (sh.W <= lds_max_bits) {
                    p->items.push_back(it);
                    ++P.n_lds;
                    P.lds_bits = std::max(P.lds_bits, sh.W);
                    P.lds_steps = std::max(P.lds_steps, sh.n_steps);
                } else {
                    hbm.push_back(it);
                    P.hbm_steps = std::max(P.hbm_steps, sh.n_steps);
                }
            }
            P.hbm0 = static_cast<int64_t>(p->hbm_entry_pre.size());
            int64_t e = 0;
            p->hbm_entry_pre.push_back(0);
            for (const TnItem &it : hbm) {
                p->items.push_back(it);
                e += 2 * (int64_t{1} << p->shapes[it.shape].W);
                p->hbm_entry_pre.push_back(e);
            }
            P.n_hbm = static_cast<int32_t>(hbm.size());
            p->n_lds += P.n_lds;
            p->n_hbm += P.n_hbm;
            p->max_items = std::max(p->max_items, P.n_lds + P.n_hbm);
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(SG_ENOMEM, "sg_tn_plan_create: host allocation");
    } catch (const std::length_error &e) {
        delete p;
        return fail(SG_EUNSUPPORTED, "sg_tn_plan_create: %s", e.what());
    }
    *out = p;
    return SG_OK;
}

int sg_tn_plan_info_get(const sg_tn_plan *p, sg_tn_plan_info *out)
{
    if (!p || !out) return fail(SG_EINVAL, "sg_tn_plan_info_get: NULL pointer");
    clear_error();
    out->L = p->L;
    out->halo = p->h;
    out->order = p->order;
    out->lds_max_bits = p->lds_bits;
    out->n_phases = static_cast<int32_t>(p->phases.size());
    out->n_shapes = static_cast<int32_t>(p->shapes.size());
    out->max_bits = p->max_bits;
    out->n_lds_sites = p->n_lds;
    out->n_hbm_sites = p->n_hbm;
    out->max_steps = p->max_steps;
    out->pair_updates = p->pair_updates;
    return SG_OK;
}

int sg_tn_plan_program(const sg_tn_plan *p, int32_t *n_shapes, int32_t *shapes, int32_t *n_steps, int32_t *steps,
                       int32_t *n_items, int32_t *items)
{
    if (!p || !n_shapes || !n_steps || !n_items) return fail(SG_EINVAL, "sg_tn_plan_program: NULL pointer");
    clear_error();
    *n_shapes = static_cast<int32_t>(p->shapes.size());
    *n_steps = static_cast<int32_t>(p->steps.size());
    *n_items = static_cast<int32_t>(p->items.size());
    if (shapes)
        for (size_t i = 0; i < p->shapes.size(); ++i) {
            const TnShape &s = p->shapes[i];
            int mask = 0;
            for (int d = 0; d < 6; ++d) mask |= (s.ccode[d] == kTnConst) << d;
            shapes[4 * i + 0] = s.W;
            shapes[4 * i + 1] = s.n_steps;
            shapes[4 * i + 2] = s.step0;
            shapes[4 * i + 3] = mask;
        }
    if (steps)
        for (size_t i = 0; i < p->steps.size(); ++i) {
            const TnStep &s = p->steps[i];
            int32_t *row = steps + 16 * i;
            row[0] = s.lv;
            row[1] = s.a;
            for (int d = 0; d < 6; ++d) row[2 + d] = s.code[d];
            row[8] = s.a_active;
            row[9] = s.n_runs;
            row[10] = s.n_base;
            row[11] = static_cast<int32_t>(s.newmask);
            for (int q = 0; q < 2; ++q) {
                uint32_t st = 0, ln = 0;
                for (int b = 0; b < 4; ++b) {
                    st |= static_cast<uint32_t>(s.run_start[4 * q + b]) << (8 * b);
                    ln |= static_cast<uint32_t>(s.run_len[4 * q + b]) << (8 * b);
                }
                row[12 + q] = static_cast<int32_t>(st);
                row[14 + q] = static_cast<int32_t>(ln);
            }
        }
    if (items)
        for (size_t i = 0; i < p->items.size(); ++i) {
            items[2 * i + 0] = p->items[i].site;
            items[2 * i + 1] = p->items[i].shape;
        }
    return SG_OK;
}

int sg_tn_plan_rounds(const sg_tn_plan *p, int32_t *n_rounds, int32_t *shape_rounds, int32_t *rounds)
{
    if (!p || !n_rounds) return fail(SG_EINVAL, "sg_tn_plan_rounds: NULL pointer");
    clear_error();
    *n_rounds = static_cast<int32_t>(p->rounds.size());
    if (shape_rounds)
        for (size_t i = 0; i < p->shapes.size(); ++i) {
            shape_rounds[2 * i + 0] = p->shapes[i].round0;
            shape_rounds[2 * i + 1] = p->shapes[i].n_rounds;
        }
    if (rounds)
        for (size_t i = 0; i < p->rounds.size(); ++i) {
            const TnRound &R = p->rounds[i];
            rounds[4 * i + 0] = R.step;   // within its shape
            rounds[4 * i + 1] = R.fused;
            rounds[4 * i + 2] = R.read_bits;
            rounds[4 * i + 3] = R.b_mode | (R.b_rank << 8);
        }
    return SG_OK;
}

}  // extern "C"
