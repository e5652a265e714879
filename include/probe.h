/*
 * probe.h -- streaming probe of the achievable HBM bandwidth of the GPU the
 * solver runs on. The solver's step is HBM-bound (each lattice update reads
 * and writes every stored population once), so its throughput is judged
 * against the nominal bandwidth and against what a plain copy, which moves
 * the same half-read, half-write mix, reaches on the same device.
 *
 * All pointers are device pointers owned by the caller; the call is queued
 * on `stream` (a hipStream_t, NULL = null stream). Nothing is allocated.
 */
#ifndef PROBE_H
#define PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PROBE_OK = 0, PROBE_EINVAL = -1, PROBE_EDEVICE = -3 };

/* dst[0 .. bytes) = src[0 .. bytes) with 16-byte accesses: blocks in
 * [1, 2^20] gives four per thread and loop trip, grid-stride over that many
 * blocks of 256 threads; blocks = 0 one per thread and no loop, as many
 * blocks as the range needs. nontemporal != 0: loads and stores carry the
 * nontemporal cache policy (the policy of the solver's stores). bytes a
 * multiple of 64, both pointers 16-byte aligned, ranges not overlapping;
 * PROBE_EINVAL otherwise. */
int probe_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal, int32_t blocks,
               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PROBE_H */
