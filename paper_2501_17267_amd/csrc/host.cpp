// host.cpp -- host-side parts of the sgmi C ABI: error reporting, beta
// schedules, acceptance tables and the synthetic tile-planted instance
// generator.  Plain C++17; no device work.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace sg {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

// Quantised acceptance probability: floor(p 2^32), saturated at 2^32-1.
static uint32_t to_u32_threshold(double p)
{
    const double scaled = std::ldexp(p, 32);
    if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
    return static_cast<uint32_t>(std::floor(scaled));
}

// ---------------------------------------------------------------------------
// splitmix64 (Steele, Lea, Flood, OOPSLA 2014)
// ---------------------------------------------------------------------------
struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t operator()()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// ---------------------------------------------------------------------------
// Tile geometry.  Corner index a = ax | ay<<1 | az<<2 of a unit cube.  The
// twelve edges are numbered x-edges 0-3 (ay + 2az), y-edges 4-7 (ax + 2az),
// z-edges 8-11 (ax + 2ay); each joins corner lo to corner lo + (1, 2 or 4).
// ---------------------------------------------------------------------------
struct EdgeTable {
    int lo[12], hi[12], axis[12];
    uint16_t face_edges[6];  // bitmask of the 4 edges of each face
    EdgeTable()
    {
        for (int e = 0; e < 12; ++e) {
            const int axis_e = e / 4, r = e % 4;
            int lo_c;
            if (axis_e == 0) lo_c = ((r & 1) << 1) | ((r >> 1) << 2);
            else if (axis_e == 1) lo_c = (r & 1) | ((r >> 1) << 2);
            else lo_c = (r & 1) | ((r >> 1) << 1);
            lo[e] = lo_c;
            hi[e] = lo_c | (1 << axis_e);
            axis[e] = axis_e;
        }
        // face (ax, side): edges whose two corners both have bit ax == side
        for (int f = 0; f < 6; ++f) {
            const int ax = f / 2, side = f % 2;
            uint16_t m = 0;
            for (int e = 0; e < 12; ++e)
                if (((lo[e] >> ax) & 1) == side && ((hi[e] >> ax) & 1) == side) m |= (uint16_t)(1u << e);
            face_edges[f] = m;
        }
    }
};
static const EdgeTable kEdges;

// number of faces whose edge-sign product is negative; `neg` has bit e set
// when coupling e is negative
static int count_frustrated(uint32_t neg)
{
    int n = 0;
    for (int f = 0; f < 6; ++f) n += __builtin_popcount(neg & kEdges.face_edges[f]) & 1;
    return n;
}

}  // namespace sg

using namespace sg;

extern "C" {

const char *sg_last_error(void) { return g_last_error.c_str(); }

const char *sg_version(void) { return "sgmi 0.1 (gfx950)"; }

const char *sg_strerror(int code)
{
    switch (code) {
    case SG_OK: return "ok";
    case SG_EINVAL: return "invalid argument";
    case SG_ENOMEM: return "out of memory";
    case SG_EDEVICE: return "device error";
    case SG_ERANGE: return "value out of range";
    case SG_EBUSY: return "resource busy";
    case SG_ENOTFOUND: return "not found";
    case SG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int sg_make_schedule(int32_t kind, double b0, double b1, int32_t S, double *beta_out)
{
    if (!beta_out) return fail(SG_EINVAL, "sg_make_schedule: beta_out is NULL");
    if (S < 1) return fail(SG_EINVAL, "sg_make_schedule: S = %d < 1", S);
    if (kind != 0 && kind != 1) return fail(SG_EINVAL, "sg_make_schedule: kind %d", kind);
    if (kind == 1 && !(b0 > 0.0 && b1 > 0.0))
        return fail(SG_EINVAL, "sg_make_schedule: geometric schedule needs positive endpoints");
    for (int32_t s = 0; s < S; ++s) {
        const double f = (S == 1) ? 0.0 : static_cast<double>(s) / static_cast<double>(S - 1);
        beta_out[s] = (kind == 0) ? b0 + (b1 - b0) * f : b0 * std::pow(b1 / b0, f);
    }
    return SG_OK;
}

int sg_make_thresholds(const double *beta, int32_t S, int32_t K, uint32_t *thr_out)
{
    if (!beta || !thr_out) return fail(SG_EINVAL, "sg_make_thresholds: NULL pointer");
    if (S < 1 || K < 1 || K > SG_K_MAX) return fail(SG_EINVAL, "sg_make_thresholds: S=%d K=%d", S, K);
    for (int32_t s = 0; s < S; ++s)
        for (int32_t k = 1; k <= K; ++k)
            thr_out[static_cast<size_t>(s) * K + (k - 1)] =
                to_u32_threshold(std::exp(-(static_cast<double>(2 * k) * beta[s])));
    return SG_OK;
}

int sg_make_exchange_thresholds(const double *beta, int32_t T, int32_t M, uint32_t *thrx_out)
{
    if (!beta || !thrx_out) return fail(SG_EINVAL, "sg_make_exchange_thresholds: NULL pointer");
    if (T < 2 || M < 1) return fail(SG_EINVAL, "sg_make_exchange_thresholds: T=%d M=%d", T, M);
    for (int32_t k = 0; k + 1 < T; ++k) {
        const double gap = beta[k + 1] - beta[k];
        for (int32_t m = 1; m <= M; ++m)
            thrx_out[static_cast<size_t>(k) * M + (m - 1)] =
                to_u32_threshold(std::exp(-(static_cast<double>(2 * m) * gap)));
    }
    return SG_OK;
}

int32_t sg_exchange_table_width(const double *beta, int32_t T)
{
    if (!beta || T < 2) return fail(SG_EINVAL, "sg_exchange_table_width: bad ladder");
    int32_t width = 1;
    for (int32_t k = 0; k + 1 < T; ++k) {
        const double gap = beta[k + 1] - beta[k];
        if (!(gap > 0.0)) return fail(SG_EINVAL, "sg_exchange_table_width: ladder not ascending");
        // largest m with floor(exp(-2 m gap) 2^32) >= 1
        int32_t m = static_cast<int32_t>(std::ceil(32.0 * std::log(2.0) / (2.0 * gap))) + 2;
        while (m > 1 && to_u32_threshold(std::exp(-(static_cast<double>(2 * m) * gap))) == 0) --m;
        if (m > width) width = m;
    }
    return width;
}

int sg_make_instance(int32_t L, int32_t cls, uint64_t seed, int8_t *J_host, int8_t *planted_host,
                     int64_t *E_gs)
{
    if (!lattice_ok(L)) return fail(SG_EINVAL, "sg_make_instance: L = %d must be even in [4, %d]", L, SG_MAX_L);
    if (!(cls == -1 || cls == 0 || cls == 2 || cls == 4 || cls == 6))
        return fail(SG_EINVAL, "sg_make_instance: class %d", cls);
    if (!J_host || !planted_host || !E_gs) return fail(SG_EINVAL, "sg_make_instance: NULL output");
    const int64_t N = static_cast<int64_t>(L) * L * L;
    auto site = [L](int x, int y, int z) -> int64_t {
        x = (x + L) % L;
        y = (y + L) % L;
        z = (z + L) % L;
        return x + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * z);
    };
    // fwd[axis][i]: coupling of the bond from site i towards +axis
    std::vector<int> fwd(3 * N, 0);
    int64_t egs = 0;
    // Tiles: cubes whose lower corner has even x+y+z.  Visiting lower
    // corners in increasing site index, the t-th tile is the one at site
    // index 2t + parity, i.e. t = i >> 1.
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = (y + z) & 1; x < L; x += 2) {
                const int64_t t = site(x, y, z) >> 1;
                SplitMix64 rng(seed ^ (static_cast<uint64_t>(t + 1) * 0xD6E8FEB86659FD93ull));
                uint32_t neg, two;
                for (;;) {
                    const uint64_t v = rng();
                    neg = static_cast<uint32_t>(v & 0xFFFu);
                    two = static_cast<uint32_t>((v >> 12) & 0xFFFu);
                    if (cls < 0 || count_frustrated(neg) == cls) break;
                }
                int Kc[12];
                for (int e = 0; e < 12; ++e) {
                    const int mag = ((two >> e) & 1u) ? 2 : 1;
                    Kc[e] = ((neg >> e) & 1u) ? -mag : mag;
                }
                // ground state of the tile: lowest energy, then lowest pattern
                int best = 0, best_E = 1 << 30;
                for (int g = 0; g < 256; ++g) {
                    int E = 0;
                    for (int e = 0; e < 12; ++e) {
                        const int sign = (((g >> kEdges.lo[e]) ^ (g >> kEdges.hi[e])) & 1) ? -1 : 1;
                        E += sign * Kc[e];
                    }
                    if (E < best_E) {
                        best_E = E;
                        best = g;
                    }
                }
                egs += best_E;
                for (int e = 0; e < 12; ++e) {
                    const int sign = (((best >> kEdges.lo[e]) ^ (best >> kEdges.hi[e])) & 1) ? -1 : 1;
                    const int a = kEdges.lo[e];
                    const int64_t p = site(x + (a & 1), y + ((a >> 1) & 1), z + ((a >> 2) & 1));
                    fwd[kEdges.axis[e] * N + p] += sign * Kc[e];
                }
            }
    // gauge: gamma_i = -1 when draw i of the gauge stream has its top bit set
    std::vector<int8_t> gamma(N);
    SplitMix64 g(seed ^ 0xA0761D6478BD642Full);
    for (int64_t i = 0; i < N; ++i) gamma[i] = (g() >> 63) ? -1 : 1;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int64_t i = site(x, y, z);
                const int64_t nb[3] = {site(x + 1, y, z), site(x, y + 1, z), site(x, y, z + 1)};
                for (int ax = 0; ax < 3; ++ax) {
                    const int v = fwd[ax * N + i] * gamma[i] * gamma[nb[ax]];
                    if (v < -4 || v > 4) return fail(SG_ERANGE, "sg_make_instance: coupling %d", v);
                    J_host[(2 * ax) * N + i] = static_cast<int8_t>(v);
                    J_host[(2 * ax + 1) * N + nb[ax]] = static_cast<int8_t>(v);
                }
            }
    std::memcpy(planted_host, gamma.data(), static_cast<size_t>(N));
    *E_gs = egs;
    return SG_OK;
}

}  // extern "C"
