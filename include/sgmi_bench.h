/*
 * sgmi_bench.h -- measurement entry points of libsgmi (not part of the
 * annealing path).
 */
#ifndef SGMI_BENCH_H
#define SGMI_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Throughput probe of one VALU instruction kind, enqueued on `stream`:
 * op 0 = v_mad_u64_u32 (the 32x32->64 product of a Philox round),
 * op 1 = 3-input xor, op 2 = 3-input add, op 3 = bitfield select.
 * blocks x 256 threads each run `iters` iterations of 8 independent
 * instructions; out: device uint32 [blocks*256] receives a checksum so the
 * work cannot be elided.  Time it with events around the call. */
int sg_microbench_valu(int32_t op, int32_t blocks, int32_t iters, uint32_t *out, void *stream);

/* Plain streaming copy of `bytes` (a multiple of 16) from src to dst (device
 * buffers): the reference kernel for converting HBM byte counters
 * (FETCH_SIZE, WRITE_SIZE) into bytes. */
int sg_microbench_copy(const void *src, void *dst, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
