// aux.hip -- energy (Eq. 1), optimality gap (Eq. 2), coupling encoding and
// instance validation kernels with their C-ABI entry points.
#include "common.hpp"
#include "sweep.hpp"
#include "variants.hpp"

namespace sg {

constexpr int kEnergyThreads = 256;

// E = sum_i s_i (J[+x][i] s_{i+x} + J[+y][i] s_{i+y} + J[+z][i] s_{i+z}):
// one work group per configuration, lanes stride over sites, wavefront
// shuffle reduction then one LDS slot per wave.
__global__ __launch_bounds__(kEnergyThreads) void k_energy(const int8_t *J, int L, const int8_t *spins,
                                                           int32_t *out)
{
    const int64_t N = static_cast<int64_t>(L) * L * L;
    const int8_t *s = spins + static_cast<int64_t>(blockIdx.x) * N;
    int32_t acc = 0;
    for (int64_t i = threadIdx.x; i < N; i += kEnergyThreads) {
        const int x = static_cast<int>(i % L);
        const int y = static_cast<int>((i / L) % L);
        const int z = static_cast<int>(i / (static_cast<int64_t>(L) * L));
        const int64_t ix = (x + 1 == L ? 0 : x + 1) + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * z);
        const int64_t iy = x + static_cast<int64_t>(L) * ((y + 1 == L ? 0 : y + 1) + static_cast<int64_t>(L) * z);
        const int64_t iz = x + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * (z + 1 == L ? 0 : z + 1));
        const int32_t si = s[i] < 0 ? -1 : 1;
        const int32_t sx = s[ix] < 0 ? -1 : 1;
        const int32_t sy = s[iy] < 0 ? -1 : 1;
        const int32_t sz = s[iz] < 0 ? -1 : 1;
        acc += si * (J[0 * N + i] * sx + J[2 * N + i] * sy + J[4 * N + i] * sz);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ int32_t part[kEnergyThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kEnergyThreads / 64; ++w) t += part[w];
        out[blockIdx.x] = t;
    }
}

__global__ void k_epsilon(const int32_t *E, int64_t n, int64_t E_gs, double *eps)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        const double gs = static_cast<double>(E_gs);
        eps[i] = static_cast<double>(static_cast<int64_t>(E[i]) - E_gs) / fabs(gs);
    }
}

// Per-group gap statistics: one work group per group of trials.  Each lane
// walks its share of the group's energies (coalesced int32 reads), keeps
// its sum, extremes and target counts in registers and adds to an LDS
// histogram; waves combine by shuffles, then one LDS slot per wave.
constexpr int kStatsThreads = 256;

struct EpsTargets {
    double t[SG_EPS_MAX_TARGETS];
};

__global__ __launch_bounds__(kStatsThreads) void k_eps_stats(const int32_t *E, int group_size, const int64_t *E_gs,
                                                             EpsTargets tg, int n_targets, double eps_max,
                                                             int n_bins, sg_eps_stats *stats, uint32_t *hist)
{
    __shared__ uint32_t s_hist[SG_EPS_MAX_BINS];
    __shared__ int64_t s_sum[kStatsThreads / 64];
    __shared__ int32_t s_min[kStatsThreads / 64], s_max[kStatsThreads / 64];
    __shared__ int32_t s_le[kStatsThreads / 64][SG_EPS_MAX_TARGETS];
    const int g = static_cast<int>(blockIdx.x);
    const int tid = static_cast<int>(threadIdx.x);
    const int32_t *e = E + static_cast<int64_t>(g) * group_size;
    const int64_t gs = E_gs[g];
    const double den = fabs(static_cast<double>(gs));
    if (hist)
        for (int b = tid; b < n_bins; b += kStatsThreads) s_hist[b] = 0u;
    __syncthreads();
    int64_t sum = 0;
    int32_t lo = 0x7FFFFFFF, hi = static_cast<int32_t>(0x80000000u);
    int32_t le[SG_EPS_MAX_TARGETS];
#pragma unroll
    for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) le[t] = 0;
    for (int i = tid; i < group_size; i += kStatsThreads) {
        const int32_t v = e[i];
        const double eps = static_cast<double>(static_cast<int64_t>(v) - gs) / den;
        sum += v;
        lo = min(lo, v);
        hi = max(hi, v);
#pragma unroll
        for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) le[t] += (t < n_targets && eps <= tg.t[t]) ? 1 : 0;
        if (hist) {
            const double pos = eps / eps_max * static_cast<double>(n_bins);
            const int b = pos < 0.0 ? 0 : (pos >= static_cast<double>(n_bins) ? n_bins - 1 : static_cast<int>(pos));
            atomicAdd(&s_hist[b], 1u);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off, 64);
        lo = min(lo, __shfl_xor(lo, off, 64));
        hi = max(hi, __shfl_xor(hi, off, 64));
#pragma unroll
        for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) le[t] += __shfl_xor(le[t], off, 64);
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
        s_sum[wave] = sum;
        s_min[wave] = lo;
        s_max[wave] = hi;
#pragma unroll
        for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) s_le[wave][t] = le[t];
    }
    __syncthreads();
    if (tid == 0) {
        sg_eps_stats out;
        out.energy_sum = 0;
        out.energy_min = 0x7FFFFFFF;
        out.energy_max = static_cast<int32_t>(0x80000000u);
        out.n = group_size;
        out.reserved = 0;
        for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) out.n_le[t] = 0;
        for (int w = 0; w < kStatsThreads / 64; ++w) {
            out.energy_sum += s_sum[w];
            out.energy_min = min(out.energy_min, s_min[w]);
            out.energy_max = max(out.energy_max, s_max[w]);
            for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) out.n_le[t] += s_le[w][t];
        }
        stats[g] = out;
    }
    if (hist)
        for (int b = tid; b < n_bins; b += kStatsThreads) hist[static_cast<int64_t>(g) * n_bins + b] = s_hist[b];
}

// Encoded couplings (HBM, dword-major so that lanes on adjacent columns
// read adjacent dwords): for colour c, direction d, half h (E = J + 8,
// F = 8 - J) and dword m, the dwords of all columns are contiguous.
template <int L>
__global__ void k_encode(const int8_t *J, uint32_t *jenc)
{
    using G = Geo<L>;
    const int total = 2 * G::NC * 6 * G::C;
    const int w = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= total) return;
    const int col = w % G::NC;   // fastest: adjacent threads write adjacent dwords
    int t = w / G::NC;
    const int m = t % G::C;
    t /= G::C;
    const int d = t % 6;
    const int c = t / 6;
    uint32_t e, f;
    encode_dword<L>(J, c, col, d, m, e, f);
    jenc[coupling_at<L, 2, kDwordMajor>(c, col, d, 0, m)] = e;
    jenc[coupling_at<L, 2, kDwordMajor>(c, col, d, 1, m)] = f;
}

__global__ void k_check(const int8_t *J, int L, int32_t *status)
{
    const int64_t N = static_cast<int64_t>(L) * L * L;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int x = static_cast<int>(i % L), y = static_cast<int>((i / L) % L);
    const int z = static_cast<int>(i / (static_cast<int64_t>(L) * L));
    int bad = 0;
    for (int d = 0; d < 6; ++d) {
        const int v = J[d * N + i];
        if (v < -4 || v > 4) ++bad;
    }
    const int64_t nx = (x + 1 == L ? 0 : x + 1) + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * z);
    const int64_t ny = x + static_cast<int64_t>(L) * ((y + 1 == L ? 0 : y + 1) + static_cast<int64_t>(L) * z);
    const int64_t nz = x + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * (z + 1 == L ? 0 : z + 1));
    if (J[0 * N + i] != J[1 * N + nx]) ++bad;
    if (J[2 * N + i] != J[3 * N + ny]) ++bad;
    if (J[4 * N + i] != J[5 * N + nz]) ++bad;
    if (bad) atomicAdd(status, bad);
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }
__global__ void k_status_finish(int32_t *p)
{
    if (*p != 0) *p = (*p > 0x3FFFFFFE) ? 0x3FFFFFFF : *p + 1;
}

static int check_launch(const char *what)
{
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "%s: launch failed: %s", what, hipGetErrorString(err));
    return SG_OK;
}

}  // namespace sg

using namespace sg;

namespace sg {

int launch_energy(const int8_t *J, int L, int n, const int8_t *spins, int32_t *out, hipStream_t stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_energy, dim3(static_cast<uint32_t>(n)), dim3(kEnergyThreads), 0, stream, J, L, spins, out);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "energy: launch failed: %s", hipGetErrorString(err));
    return SG_OK;
}

}  // namespace sg

extern "C" {

int energy(const sg_instance *inst, int32_t n_rep, const int8_t *spins, int32_t *energy_out, void *stream)
{
    if (!inst || !inst->J || !spins || !energy_out) return fail(SG_EINVAL, "energy: NULL pointer");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "energy: L = %d", inst->L);
    if (n_rep < 1) return fail(SG_EINVAL, "energy: n_rep = %d", n_rep);
    clear_error();
    return launch_energy(inst->J, inst->L, n_rep, spins, energy_out, static_cast<hipStream_t>(stream));
}

int epsilon(const int32_t *energy_in, int64_t n, int64_t E_gs, double *eps_out, void *stream)
{
    if (!energy_in || !eps_out) return fail(SG_EINVAL, "epsilon: NULL pointer");
    if (n < 1) return fail(SG_EINVAL, "epsilon: n = %lld", static_cast<long long>(n));
    if (E_gs == 0) return fail(SG_EINVAL, "epsilon: E_gs must be nonzero");
    clear_error();
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_epsilon, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0,
                       static_cast<hipStream_t>(stream), energy_in, n, E_gs, eps_out);
    return check_launch("epsilon");
}

int epsilon_stats(const int32_t *energy_in, int32_t n_groups, int32_t group_size, const int64_t *E_gs,
                  const double *targets, int32_t n_targets, double eps_max, int32_t n_bins, sg_eps_stats *stats_out,
                  uint32_t *hist_out, void *stream)
{
    if (!energy_in || !E_gs || !stats_out) return fail(SG_EINVAL, "epsilon_stats: NULL energy, E_gs or stats_out");
    if (n_groups < 1 || group_size < 1)
        return fail(SG_EINVAL, "epsilon_stats: n_groups = %d, group_size = %d", n_groups, group_size);
    if (n_targets < 0 || n_targets > SG_EPS_MAX_TARGETS || (n_targets > 0 && !targets))
        return fail(SG_EINVAL, "epsilon_stats: n_targets = %d (0..%d, targets[] given)", n_targets,
                    SG_EPS_MAX_TARGETS);
    if (hist_out && (n_bins < 1 || n_bins > SG_EPS_MAX_BINS || !(eps_max > 0.0)))
        return fail(SG_EINVAL, "epsilon_stats: histogram needs 1 <= n_bins <= %d and eps_max > 0", SG_EPS_MAX_BINS);
    EpsTargets tg;
    for (int t = 0; t < SG_EPS_MAX_TARGETS; ++t) tg.t[t] = t < n_targets ? targets[t] : 0.0;
    clear_error();
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_eps_stats, dim3(static_cast<unsigned>(n_groups)), dim3(kStatsThreads), 0,
                       static_cast<hipStream_t>(stream), energy_in, group_size, E_gs, tg, n_targets,
                       hist_out ? eps_max : 1.0, hist_out ? n_bins : 0, stats_out, hist_out);
    return check_launch("epsilon_stats");
}

size_t sg_jenc_bytes(int32_t L)
{
    if (!lattice_ok(L)) return 0;
    const size_t H = L / 2, NC = H * L, C = (L + 3) / 4;
    return 2 * NC * 6 * 2 * C * sizeof(uint32_t);
}

int sg_encode_instance(const sg_instance *inst, uint32_t *jenc_out, void *stream)
{
    if (!inst || !inst->J || !jenc_out) return fail(SG_EINVAL, "sg_encode_instance: NULL pointer");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "sg_encode_instance: L = %d", inst->L);
    clear_error();
    const int64_t total = static_cast<int64_t>(sg_jenc_bytes(inst->L) / sizeof(uint32_t) / 2);
    const int threads = 256;
    const dim3 grid(static_cast<unsigned>((total + threads - 1) / threads));
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    switch (inst->L) {
#define SG_ENC(LL) \
    case LL: hipLaunchKernelGGL(k_encode<LL>, grid, dim3(threads), 0, st, inst->J, jenc_out); break;
        SG_ENC(4) SG_ENC(6) SG_ENC(8) SG_ENC(10) SG_ENC(12) SG_ENC(14) SG_ENC(16) SG_ENC(18) SG_ENC(20)
        SG_ENC(22) SG_ENC(24) SG_ENC(26) SG_ENC(28) SG_ENC(30) SG_ENC(32) SG_ENC(34) SG_ENC(36) SG_ENC(38)
        SG_ENC(40) SG_ENC(42) SG_ENC(44) SG_ENC(46) SG_ENC(48) SG_ENC(50) SG_ENC(52) SG_ENC(54) SG_ENC(56)
        SG_ENC(58) SG_ENC(60) SG_ENC(62) SG_ENC(64)
#undef SG_ENC
    default: return fail(SG_EINVAL, "sg_encode_instance: L = %d", inst->L);
    }
    return check_launch("sg_encode_instance");
}

int sg_check_instance(const sg_instance *inst, int32_t *status_out, void *stream)
{
    if (!inst || !inst->J || !status_out) return fail(SG_EINVAL, "sg_check_instance: NULL pointer");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "sg_check_instance: L = %d", inst->L);
    clear_error();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t N = static_cast<int64_t>(inst->L) * inst->L * inst->L;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, st, status_out, 0);
    hipLaunchKernelGGL(k_check, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, st, inst->J, inst->L,
                       status_out);
    hipLaunchKernelGGL(k_status_finish, dim3(1), dim3(1), 0, st, status_out);
    return check_launch("sg_check_instance");
}

}  // extern "C"
