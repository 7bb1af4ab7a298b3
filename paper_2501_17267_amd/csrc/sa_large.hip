// sa_large.hip -- annealing kernels of the lattice sizes between 32 and 64
// (L = 34 .. 62): couplings streamed from the encoded image and spins in the
// caller's workspace, one replica per work group, as at L = 64.  These are
// the sizes of the paper's scaling study of simulated annealing (App. D);
// they live in their own translation unit so that the library compiles in
// parallel.
#include "sa_launch.hpp"

namespace sg {

#define SG_VL(LL) \
    static const SaVariant kVL##LL[] = {SG_VX(LL, 1, 16, kJGlobalEF, false), SG_VX(LL, 1, 8, kJGlobalEF, false)};
SG_VL(34) SG_VL(36) SG_VL(38) SG_VL(40) SG_VL(42) SG_VL(44) SG_VL(46) SG_VL(48)
SG_VL(50) SG_VL(52) SG_VL(54) SG_VL(56) SG_VL(58) SG_VL(60) SG_VL(62)
#undef SG_VL
#undef SG_V
#undef SG_VX

const SaVariant *sa_variants_large(int L, int *n)
{
#define SG_CASE(LL)                                                  \
    case LL:                                                         \
        *n = static_cast<int>(sizeof(kVL##LL) / sizeof(kVL##LL[0])); \
        return kVL##LL;
    switch (L) {
        SG_CASE(34) SG_CASE(36) SG_CASE(38) SG_CASE(40) SG_CASE(42) SG_CASE(44) SG_CASE(46) SG_CASE(48)
        SG_CASE(50) SG_CASE(52) SG_CASE(54) SG_CASE(56) SG_CASE(58) SG_CASE(60) SG_CASE(62)
    default:
        *n = 0;
        return nullptr;
    }
#undef SG_CASE
}

}  // namespace sg
