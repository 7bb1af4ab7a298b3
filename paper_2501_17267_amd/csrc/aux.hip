// aux.hip -- energy (Eq. 1), optimality gap (Eq. 2), coupling encoding and
// instance validation kernels with their C-ABI entry points.
#include "common.hpp"
#include "device.hpp"

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

// Encoded couplings: for colour c, column col, direction d, dword m the E
// (J + 8) and F (8 - J) bytes of the four sites z = 4m .. 4m+3.
__global__ void k_encode(const int8_t *J, int L, uint32_t *jenc)
{
    const int H = L / 2, NC = H * L, C = (L + 3) / 4;
    const int64_t N = static_cast<int64_t>(L) * L * L;
    const int64_t total = static_cast<int64_t>(2) * NC * 6 * C;
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= total) return;
    const int m = static_cast<int>(w % C);
    int64_t t = w / C;
    const int d = static_cast<int>(t % 6);
    t /= 6;
    const int col = static_cast<int>(t % NC);
    const int c = static_cast<int>(t / NC);
    const int k = col % H, y = col / H;
    uint32_t e = 0, f = 0;
    for (int b = 0; b < 4; ++b) {
        const int z = 4 * m + b;
        int jv = 0;
        if (z < L) {
            const int x = 2 * k + ((y + z + c) & 1);
            jv = J[d * N + x + static_cast<int64_t>(L) * (y + static_cast<int64_t>(L) * z)];
        }
        e |= static_cast<uint32_t>(8 + jv) << (8 * b);
        f |= static_cast<uint32_t>(8 - jv) << (8 * b);
    }
    const int64_t base = (static_cast<int64_t>(c) * NC + col) * 6 + d;
    jenc[base * 2 * C + m] = e;
    jenc[base * 2 * C + C + m] = f;
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

extern "C" {

int energy(const sg_instance *inst, int32_t n_rep, const int8_t *spins, int32_t *energy_out, void *stream)
{
    if (!inst || !inst->J || !spins || !energy_out) return fail(SG_EINVAL, "energy: NULL pointer");
    if (!lattice_ok(inst->L)) return fail(SG_EINVAL, "energy: L = %d", inst->L);
    if (n_rep < 1) return fail(SG_EINVAL, "energy: n_rep = %d", n_rep);
    clear_error();
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_energy, dim3(n_rep), dim3(kEnergyThreads), 0, static_cast<hipStream_t>(stream),
                       inst->J, inst->L, spins, energy_out);
    return check_launch("energy");
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
    const int64_t total = static_cast<int64_t>(sg_jenc_bytes(inst->L) / sizeof(uint32_t));
    const int threads = 256;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_encode, dim3(static_cast<unsigned>((total + threads - 1) / threads)), dim3(threads), 0,
                       static_cast<hipStream_t>(stream), inst->J, inst->L, jenc_out);
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
