// microbench.hip -- throughput probes of the VALU instructions the annealing
// kernels are built from (32x32->64 multiply-add, 3-input xor, 3-input add,
// bitfield select), used to state the ALU ceiling of the sweep kernels with
// measured rather than assumed instruction costs.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "sgmi_bench.h"

namespace sg {

constexpr int kChains = 8;

template <int OP>
__global__ __launch_bounds__(256) void k_probe(uint32_t *out, int iters, uint32_t seed)
{
    uint32_t a[kChains];
    uint64_t p[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = seed * (threadIdx.x + 1) + c;
        p[c] = a[c] ^ 0x5555u;
    }
    uint32_t k = seed;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (OP == 0) {  // v_mad_u64_u32
                p[c] = static_cast<uint64_t>(static_cast<uint32_t>(p[c])) * 0xD2511F53u + p[c];
            } else if (OP == 1) {  // v_xor3_b32
                a[c] = a[c] ^ a[(c + 1) % kChains] ^ k;
            } else if (OP == 2) {  // v_add3_u32
                a[c] = a[c] + a[(c + 1) % kChains] + k;
            } else {  // bitfield select
                a[c] = (a[c] & a[(c + 1) % kChains]) | (~a[c] & k);
            }
        }
        k += 0x9E3779B9u;
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= a[c] ^ static_cast<uint32_t>(p[c]) ^ static_cast<uint32_t>(p[c] >> 32);
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// plain streaming copy of n 16-byte words (the reference for scaling the
// HBM byte counters)
__global__ __launch_bounds__(256) void k_copy(const uint4 *src, uint4 *dst, int64_t n)
{
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256)
        dst[i] = src[i];
}

}  // namespace sg

using namespace sg;

extern "C" int sg_microbench_copy(const void *src, void *dst, int64_t bytes, void *stream)
{
    if (!src || !dst || bytes < 16 || (bytes % 16) != 0) return fail(SG_EINVAL, "sg_microbench_copy: bad arguments");
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_copy, dim3(256 * 8), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), bytes / 16);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_microbench_copy: %s", hipGetErrorString(err));
    return SG_OK;
}

extern "C" int sg_microbench_valu(int32_t op, int32_t blocks, int32_t iters, uint32_t *out, void *stream)
{
    if (op < 0 || op > 3 || blocks < 1 || iters < 1 || !out) return fail(SG_EINVAL, "sg_microbench_valu: bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    switch (op) {
    case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, st, out, iters, 12345u); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, st, out, iters, 12345u); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, st, out, iters, 12345u); break;
    default: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, st, out, iters, 12345u); break;
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_microbench_valu: %s", hipGetErrorString(err));
    return SG_OK;
}
