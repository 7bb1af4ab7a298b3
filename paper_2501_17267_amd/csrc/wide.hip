// wide.hip -- simulated annealing of a few replicas of a large lattice
// (L above the LDS-resident sizes) spread over the whole device.
//
// The single-work-group kernels give one replica one compute unit.  Here
// each colour phase of each sweep is one launch with one lane per column
// dword of every replica; the boundary between two launches is the barrier
// between the phases, so no work group ever waits on another.  Spins live
// in the caller's workspace in the dword-major column layout, couplings are
// read from the encoded image; the Philox counters, tables and acceptance
// are those of the single-work-group kernels, so results are identical.
#include "common.hpp"
#include "variants.hpp"

namespace sg {

constexpr int kWideThreads = 256;

template <int L>
using WideCol = Column<L, true, kDwordMajor, kDwordMajor>;

// Initial column-layout spins of every replica, one lane per dword: from
// the init stream (site i draws word i mod 4 of call floor(i/4)) or from the
// caller's natural-order spins.  Padding bytes (L = 2 mod 4) are zero.
template <int L>
__global__ __launch_bounds__(kWideThreads) void k_wide_init(SaJob job)
{
    using G = Geo<L>;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kWideThreads + threadIdx.x;
    if (t >= static_cast<int64_t>(job.n_rep) * G::SPIN_DW) return;
    const int r = static_cast<int>(t / G::SPIN_DW);
    const int rem = static_cast<int>(t - static_cast<int64_t>(r) * G::SPIN_DW);
    // dword-major: rem = (c*C + m)*NC + col
    const int col = rem % G::NC;
    const int cm = rem / G::NC;
    const int m = cm % G::C;
    const int c = cm / G::C;
    const int k = col % G::H;
    const int y = col / G::H;
    const uint32_t rep_word = job.rep0 + static_cast<uint32_t>(r);
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int z = 4 * m + b;
        if (z >= L) continue;
        const int x = 2 * k + ((y + z + c) & 1);
        const int i = x + L * (y + L * z);
        bool neg;
        if (job.init_random) {
            const Rand4 u = philox10(static_cast<uint32_t>(i >> 2), 0xFFFFFFFFu, rep_word, job.chain, job.k0, job.k1);
            const uint32_t word = (i & 3) == 0 ? u.w[0] : (i & 3) == 1 ? u.w[1] : (i & 3) == 2 ? u.w[2] : u.w[3];
            neg = (word >> 31) != 0;
        } else {
            neg = job.spins[static_cast<int64_t>(r) * G::N + i] < 0;
        }
        if (neg) w |= 0xFFu << (8 * b);
    }
    job.workspace[t] = w;
    if (rem == 0) job.energy[r] = 0;   // accumulated by k_wide_final
}

// One colour phase of sweep si (row si of the thresholds): lane = dword m of
// column col of colour c of replica r; consecutive lanes take consecutive
// columns, so spin and coupling loads coalesce.
template <int L>
__global__ __launch_bounds__(kWideThreads) void k_wide_phase(SaJob job, int si, int c)
{
    using G = Geo<L>;
    __shared__ uint32_t tb[kThrEntries];
    if (threadIdx.x < kThrEntries)
        tb[threadIdx.x] = thr_entry(job.thr + static_cast<int64_t>(si) * job.K, job.K, static_cast<int>(threadIdx.x));
    __syncthreads();
    constexpr int PER = G::NC * G::C;  // dwords of one colour of one replica
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kWideThreads + threadIdx.x;
    if (t >= static_cast<int64_t>(job.n_rep) * PER) return;
    const int r = static_cast<int>(t / PER);
    const int rem = static_cast<int>(t - static_cast<int64_t>(r) * PER);
    const int m = rem / G::NC;
    const int col = rem - m * G::NC;
    uint32_t *rep = job.workspace + static_cast<int64_t>(r) * G::SPIN_DW;
    const int at = spin_at<L, kDwordMajor>(c, col, m);
    const uint32_t own = rep[at];
    const uint32_t kbm = WideCol<L>::field_dword(rep, job.jenc, c, col, m, own);
    const uint32_t s_abs = static_cast<uint32_t>(job.sweep0 + si);
    const Rand4 u = philox10(static_cast<uint32_t>(col * G::C + m), 2u * s_abs + static_cast<uint32_t>(c),
                             job.rep0 + static_cast<uint32_t>(r), job.chain, job.k0, job.k1);
    int32_t dE = 0;
    rep[at] = own ^ WideCol<L>::template accept_dword<false>(kbm, u, reinterpret_cast<const char *>(tb), m, dE);
}

// Natural-order spins back to the caller and the energy of Eq. 1 (the sum
// over colour-0 sites of s_i h_i), kWideFinalGroups work groups per replica,
// each on a slice of the quads and colour-0 dwords; the energy (zeroed by
// k_wide_init) accumulates atomically.
constexpr int kWideFinalGroups = 64;

template <int L>
__global__ __launch_bounds__(kWideThreads) void k_wide_final(SaJob job)
{
    using G = Geo<L>;
    const int r = static_cast<int>(blockIdx.x) / kWideFinalGroups;
    const int part = static_cast<int>(blockIdx.x) - r * kWideFinalGroups;
    const int tid = static_cast<int>(threadIdx.x);
    const uint32_t *rep = job.workspace + static_cast<int64_t>(r) * G::SPIN_DW;
    const uint8_t *repb = reinterpret_cast<const uint8_t *>(rep);
    constexpr int QN = G::N / 4, QP = (QN + kWideFinalGroups - 1) / kWideFinalGroups;
    for (int q = part * QP + tid; q < min(QN, (part + 1) * QP); q += kWideThreads)
        store_spins_one<L, kDwordMajor>(repb, q, job.spins + static_cast<int64_t>(r) * G::N);
    constexpr int WN = G::C * G::NC, WP = (WN + kWideFinalGroups - 1) / kWideFinalGroups;
    int32_t e = 0;
    for (int w = part * WP + tid; w < min(WN, (part + 1) * WP); w += kWideThreads) {
        const int m = w / G::NC;
        const int col = w - m * G::NC;
        const uint32_t own = rep[spin_at<L, kDwordMajor>(0, col, m)];
        const uint32_t kbm = WideCol<L>::field_dword(rep, job.jenc, 0, col, m, own);
        const int nvalid = (G::TAIL != 0 && m == G::C - 1) ? G::TAIL : 4;
        e += static_cast<int32_t>(kKbBias) * nvalid -
             static_cast<int32_t>(byte_sum(kbm & WideCol<L>::valid(m)));
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    __shared__ int32_t partial[kWideThreads / 64];
    if ((tid & 63) == 0) partial[tid >> 6] = e;
    __syncthreads();
    if (tid == 0) {
        int32_t total = 0;
        for (int i = 0; i < kWideThreads / 64; ++i) total += partial[i];
        if (total != 0) atomicAdd(&job.energy[r], total);
    }
}

template <int L>
static int launch_wide(const SaJob &job, hipStream_t st)
{
    using G = Geo<L>;
    (void)hipGetLastError();
    const int64_t n_init = static_cast<int64_t>(job.n_rep) * G::SPIN_DW;
    hipLaunchKernelGGL(k_wide_init<L>, dim3(static_cast<uint32_t>((n_init + kWideThreads - 1) / kWideThreads)),
                       dim3(kWideThreads), 0, st, job);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sa_anneal (wide): launch failed: %s", hipGetErrorString(err));
    const int64_t n_phase = static_cast<int64_t>(job.n_rep) * G::NC * G::C;
    const dim3 grid(static_cast<uint32_t>((n_phase + kWideThreads - 1) / kWideThreads));
    for (int si = 0; si < job.n_sweeps; ++si)
        for (int c = 0; c < 2; ++c) hipLaunchKernelGGL(k_wide_phase<L>, grid, dim3(kWideThreads), 0, st, job, si, c);
    hipLaunchKernelGGL(k_wide_final<L>, dim3(static_cast<uint32_t>(job.n_rep) * kWideFinalGroups),
                       dim3(kWideThreads), 0, st, job);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sa_anneal (wide): launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

bool wide_supported(int L) { return L > SG_LDS_MAX_L && lattice_ok(L); }

size_t wide_bytes(int L, int n_rep)
{
    const size_t H = L / 2, NC = H * L, C = (L + 3) / 4;
    return static_cast<size_t>(n_rep) * 2 * NC * C * sizeof(uint32_t);
}

int sa_wide(const SaJob &job, int L, hipStream_t st)
{
    switch (L) {
    case 26: return launch_wide<26>(job, st);
    case 28: return launch_wide<28>(job, st);
    case 30: return launch_wide<30>(job, st);
    case 32: return launch_wide<32>(job, st);
    case 34: return launch_wide<34>(job, st);
    case 36: return launch_wide<36>(job, st);
    case 38: return launch_wide<38>(job, st);
    case 40: return launch_wide<40>(job, st);
    case 42: return launch_wide<42>(job, st);
    case 44: return launch_wide<44>(job, st);
    case 46: return launch_wide<46>(job, st);
    case 48: return launch_wide<48>(job, st);
    case 50: return launch_wide<50>(job, st);
    case 52: return launch_wide<52>(job, st);
    case 54: return launch_wide<54>(job, st);
    case 56: return launch_wide<56>(job, st);
    case 58: return launch_wide<58>(job, st);
    case 60: return launch_wide<60>(job, st);
    case 62: return launch_wide<62>(job, st);
    case 64: return launch_wide<64>(job, st);
    default: return fail(SG_EUNSUPPORTED, "sa_anneal (wide): L = %d", L);
    }
}

}  // namespace sg
