// host_checks.cpp -- host code of the library built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitized.py builds and runs
// it): the instance generator, schedules and threshold tables (host.cpp),
// the tensor-network planner (tn_plan.cpp), and the anneal server's
// admission policy (admission.hpp) driven by a scripted clock.  Exits 0 when
// every check holds; any sanitizer report aborts with a nonzero status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <set>
#include <vector>

#include "admission.hpp"
#include "sgmi.h"
#include "tn.hpp"

static int g_failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_failures;                                               \
        }                                                               \
    } while (0)

using sg::AdmitCapacity;
using sg::AdmitEntry;

static std::vector<uint64_t> ids(const std::vector<AdmitEntry> &v)
{
    std::vector<uint64_t> out;
    for (const auto &e : v) out.push_back(e.id);
    return out;
}

static void admission_checks()
{
    const auto none = [](uint64_t) { return false; };
    const double age = 0.05;
    // everything fits: arrival order
    {
        std::deque<AdmitEntry> q{{1, 100, false, 0.0}, {2, 100, false, 0.0}, {3, 100, false, 0.0}};
        AdmitCapacity cap{0, 10, 0, 1000, 0};
        auto got = ids(sg::admit_pick(q, cap, 0.0, age, none));
        CHECK((got == std::vector<uint64_t>{1, 2, 3}) && q.empty());
        CHECK(cap.active == 3 && cap.mem_in_use == 300);
    }
    // the active limit stops admission; the rest stay queued in order
    {
        std::deque<AdmitEntry> q{{1, 1, false, 0}, {2, 1, false, 0}, {3, 1, false, 0}};
        AdmitCapacity cap{1, 2, 0, 1000, 0};
        auto got = ids(sg::admit_pick(q, cap, 0.0, age, none));
        CHECK((got == std::vector<uint64_t>{1}) && q.size() == 2 && q.front().id == 2);
    }
    // a young large request without a free workspace is passed over by the
    // small ones behind it
    {
        std::deque<AdmitEntry> q{{1, 500, true, 1.00}, {2, 10, false, 1.01}, {3, 10, false, 1.02}};
        AdmitCapacity cap{0, 10, 0, 1000, 0};
        auto got = ids(sg::admit_pick(q, cap, 1.03, age, none));
        CHECK((got == std::vector<uint64_t>{2, 3}) && q.size() == 1 && q.front().id == 1);
        // later, old: it holds back what arrives behind it
        q.push_back({4, 10, false, 1.20});
        got = ids(sg::admit_pick(q, cap, 1.00 + age, age, none));
        CHECK(got.empty() && q.size() == 2);
        // a workspace frees: it goes first, then the one behind it
        cap.ws_free = 1;
        got = ids(sg::admit_pick(q, cap, 1.30, age, none));
        CHECK((got == std::vector<uint64_t>{1, 4}) && q.empty() && cap.ws_free == 0);
    }
    // the memory budget: a request too big for what is left is passed over
    // while young; a smaller one behind it fits
    {
        std::deque<AdmitEntry> q{{7, 600, false, 5.0}, {8, 300, false, 5.0}};
        AdmitCapacity cap{1, 10, 500, 1000, 0};
        auto got = ids(sg::admit_pick(q, cap, 5.01, age, none));
        CHECK((got == std::vector<uint64_t>{8}) && cap.mem_in_use == 800 && q.front().id == 7);
        cap.mem_in_use = 300;   // requests retired
        got = ids(sg::admit_pick(q, cap, 5.02, age, none));
        CHECK((got == std::vector<uint64_t>{7}) && q.empty());
    }
    // cancelled entries are dropped wherever they are
    {
        std::deque<AdmitEntry> q{{1, 1, false, 0}, {2, 1, false, 0}, {3, 1, false, 0}};
        AdmitCapacity cap{0, 10, 0, 1000, 0};
        auto got = ids(sg::admit_pick(q, cap, 0.0, age, [](uint64_t id) { return id == 2; }));
        CHECK((got == std::vector<uint64_t>{1, 3}) && q.empty());
    }
    // a scripted stream: nothing is admitted twice, every request eventually
    // is, and no request waits past the age bound while a later one that
    // arrived after it became old is admitted
    {
        std::deque<AdmitEntry> q;
        AdmitCapacity cap{0, 8, 0, 4000, 2};
        std::set<uint64_t> seen;
        std::vector<std::pair<double, AdmitEntry>> live;   // admitted: (retire time, entry)
        uint64_t next = 1;
        for (int tick = 0; tick < 4000; ++tick) {
            const double now = tick * 0.001;
            if (tick < 3000 && tick % 3 == 0) {
                const bool big = (next % 11) == 0;
                q.push_back({next, big ? 1500 : 100, big, now});
                ++next;
            }
            for (size_t i = 0; i < live.size();) {
                if (live[i].first <= now) {
                    cap.active -= 1;
                    cap.mem_in_use -= live[i].second.footprint;
                    if (live[i].second.needs_ws) cap.ws_free += 1;
                    live.erase(live.begin() + static_cast<long>(i));
                } else {
                    ++i;
                }
            }
            for (const AdmitEntry &e : sg::admit_pick(q, cap, now, age, none)) {
                CHECK(seen.insert(e.id).second);
                live.push_back({now + (e.needs_ws ? 0.030 : 0.010), e});
            }
            CHECK(cap.active <= 8 && cap.mem_in_use <= 4000 && cap.ws_free >= 0);
        }
        CHECK(q.empty() && seen.size() == next - 1);
    }
}

static void generator_and_table_checks()
{
    for (int L : {4, 6, 10}) {
        const int N = L * L * L;
        std::vector<int8_t> J(6 * N), g(N);
        int64_t egs = 0;
        CHECK(sg_make_instance(L, 6, 1234 + L, J.data(), g.data(), &egs) == SG_OK);
        CHECK(egs < 0);
        int64_t e = 0;
        for (int i = 0; i < N; ++i) {
            const int x = i % L, y = (i / L) % L, z = i / (L * L);
            const int nx = (x + 1) % L + L * (y + L * z), ny = x + L * ((y + 1) % L + L * z),
                      nz = x + L * (y + L * ((z + 1) % L));
            e += g[i] * (J[0 * N + i] * g[nx] + J[2 * N + i] * g[ny] + J[4 * N + i] * g[nz]);
            CHECK(J[0 * N + i] == J[1 * N + nx] && J[2 * N + i] == J[3 * N + ny] && J[4 * N + i] == J[5 * N + nz]);
        }
        CHECK(e == egs);
    }
    std::vector<int8_t> J(6 * 64), g(64);
    int64_t egs = 0;
    CHECK(sg_make_instance(5, 6, 1, J.data(), g.data(), &egs) == SG_EINVAL);
    CHECK(sg_make_instance(4, 3, 1, J.data(), g.data(), &egs) == SG_EINVAL);
    std::vector<double> beta(7);
    CHECK(sg_make_schedule(1, 0.2, 3.0, 7, beta.data()) == SG_OK);
    CHECK(std::fabs(beta[0] - 0.2) < 1e-15 && std::fabs(beta[6] - 3.0) < 1e-12);
    CHECK(sg_make_schedule(2, 0.2, 3.0, 7, beta.data()) == SG_EINVAL);
    std::vector<uint32_t> thr(7 * SG_K_MAX);
    CHECK(sg_make_thresholds(beta.data(), 7, SG_K_MAX, thr.data()) == SG_OK);
    for (int s = 0; s < 7; ++s)
        for (int k = 1; k < SG_K_MAX; ++k) CHECK(thr[s * SG_K_MAX + k] <= thr[s * SG_K_MAX + k - 1]);
    const int M = sg_exchange_table_width(beta.data(), 7);
    CHECK(M >= 1);
    std::vector<uint32_t> thrx(6 * M);
    CHECK(sg_make_exchange_thresholds(beta.data(), 7, M, thrx.data()) == SG_OK);
    CHECK(sg_make_thresholds(beta.data(), 7, SG_K_MAX + 1, thr.data()) != SG_OK);
    CHECK(sg_strerror(SG_EINVAL) != nullptr && sg_last_error() != nullptr);
}

static void planner_checks()
{
    struct Case {
        int L, h, order, bits;
    };
    for (const Case &c : {Case{6, 1, 0, 0}, Case{6, 1, 1, 4}, Case{10, 2, 1, 0}, Case{6, 2, 0, 8}}) {
        sg_tn_plan *p = nullptr;
        CHECK(sg_tn_plan_create(c.L, c.h, c.order, c.bits, &p) == SG_OK && p);
        if (!p) continue;
        sg_tn_plan_info info{};
        CHECK(sg_tn_plan_info_get(p, &info) == SG_OK);
        CHECK(info.n_lds_sites + info.n_hbm_sites == c.L * c.L * c.L);
        int32_t ns = 0, nt = 0, ni = 0;
        CHECK(sg_tn_plan_program(p, &ns, nullptr, &nt, nullptr, &ni, nullptr) == SG_OK);
        std::vector<int32_t> shapes(4 * ns), steps(16 * nt), items(2 * ni);
        CHECK(sg_tn_plan_program(p, &ns, shapes.data(), &nt, steps.data(), &ni, items.data()) == SG_OK);
        CHECK(ni == c.L * c.L * c.L);
        std::set<int32_t> sites;
        for (int i = 0; i < ni; ++i) {
            sites.insert(items[2 * i]);
            CHECK(items[2 * i + 1] >= 0 && items[2 * i + 1] < ns);
        }
        CHECK(static_cast<int>(sites.size()) == ni);
        for (int s = 0; s < ns; ++s) CHECK(shapes[4 * s + 2] + shapes[4 * s + 1] <= nt);
        delete p;   // no device copy exists before a first decimation
    }
    sg_tn_plan *p = nullptr;
    CHECK(sg_tn_plan_create(6, 3, 1, 0, &p) == SG_EINVAL && !p);
    CHECK(sg_tn_plan_create(7, 1, 1, 0, &p) == SG_EINVAL && !p);
}

int main()
{
    admission_checks();
    generator_and_table_checks();
    planner_checks();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
