// Streaming copy probe (include/probe.h): the achievable HBM bandwidth of a
// half-read, half-write stream, the traffic mix of the solver's step.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "probe.h"

namespace {

// Discards an error that an earlier HIP call of another library left pending
// in this thread, so that the check after an entry point's launches
// (hipGetLastError) reports only that entry point's own failures.
inline void clear_stale_error() { (void)hipGetLastError(); }


typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Four 16-byte values per thread and trip: the four loads are issued before
// the first store, so each wavefront keeps 4 KiB in flight.
template <bool NT>
__global__ void __launch_bounds__(256) copy_kernel(const u32x4 *__restrict__ src,
                                                   u32x4 *__restrict__ dst, size_t n4) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32x4 *p = src + i + k * n4;
            v[k] = NT ? __builtin_nontemporal_load(p) : *p;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            u32x4 *q = dst + i + k * n4;
            if (NT) __builtin_nontemporal_store(v[k], q);
            else *q = v[k];
        }
    }
}

// One 16-byte value per thread, no loop: as many blocks as the range needs.
// Each wavefront issues its load, and the store behind it, once; the chip
// is filled by the number of wavefronts in flight rather than by trips of a
// loop (measured the fastest form of a plain copy on gfx950).
template <bool NT>
__global__ void __launch_bounds__(256) copy1_kernel(const u32x4 *__restrict__ src,
                                                    u32x4 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const u32x4 v = NT ? __builtin_nontemporal_load(src + i) : src[i];
    if (NT) __builtin_nontemporal_store(v, dst + i);
    else dst[i] = v;
}

}  // namespace

extern "C" int probe_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal,
                          int32_t blocks, void *stream) {
    clear_stale_error();
    if (!src || !dst || bytes == 0 || bytes % 64 != 0 || blocks < 0 || blocks > (1 << 20))
        return PROBE_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return PROBE_EINVAL;
    const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
    if (s0 < d0 + bytes && d0 < s0 + bytes) return PROBE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (blocks == 0) {
        const size_t n = bytes / 16, nb = (n + 255) / 256;
        if (nb > 0x7fffffffu) return PROBE_EINVAL;
        if (nontemporal)
            hipLaunchKernelGGL(copy1_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st,
                               (const u32x4 *)src, (u32x4 *)dst, n);
        else
            hipLaunchKernelGGL(copy1_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st,
                               (const u32x4 *)src, (u32x4 *)dst, n);
        return hipGetLastError() == hipSuccess ? PROBE_OK : PROBE_EDEVICE;
    }
    // the range is split in four quarters; thread i copies element i of each
    const size_t n4 = bytes / 64;
    if (nontemporal)
        hipLaunchKernelGGL(copy_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const u32x4 *)src, (u32x4 *)dst, n4);
    else
        hipLaunchKernelGGL(copy_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const u32x4 *)src, (u32x4 *)dst, n4);
    return hipGetLastError() == hipSuccess ? PROBE_OK : PROBE_EDEVICE;
}
