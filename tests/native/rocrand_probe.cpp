// rocrand_probe.cpp -- test helper: evaluates Philox4x32-10 with rocRAND's
// open-source host/device engine (rocrand/rocrand_philox4x32_10.h), an
// implementation independent of both the oracle and the HIP kernels.  Host
// code only; nothing here launches a kernel.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>

namespace {
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};
}  // namespace

extern "C" void rocrand_philox_blocks(const uint32_t *ctr, uint32_t k0, uint32_t k1,
                                      uint32_t *out, int64_t n)
{
    Probe p;
    uint2 key;
    key.x = k0;
    key.y = k1;
    for (int64_t i = 0; i < n; ++i) {
        uint4 c;
        c.x = ctr[4 * i + 0];
        c.y = ctr[4 * i + 1];
        c.z = ctr[4 * i + 2];
        c.w = ctr[4 * i + 3];
        uint4 r = p.block(c, key);
        out[4 * i + 0] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}

// The public engine interface: seed, subsequence (counter words 2-3) and
// offset (4 x counter words 0-1), then four draws.  Valid for counters with
// word 1 below 2^30 so that the 64-bit offset does not overflow.
extern "C" void rocrand_philox_public(uint64_t seed, const uint32_t *ctr, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        unsigned long long sub = (unsigned long long)ctr[4 * i + 2] |
                                 ((unsigned long long)ctr[4 * i + 3] << 32);
        unsigned long long off = 4ull * ((unsigned long long)ctr[4 * i + 0] |
                                         ((unsigned long long)ctr[4 * i + 1] << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = e.next();
    }
}
