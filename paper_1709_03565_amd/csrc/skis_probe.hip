// skis_probe.hip -- random-read bandwidth probe: the achievable HBM bandwidth of uniformly
// random reads of one row size, the ceiling against which the sampler's random-access
// kernels are measured (they read 8-byte row bounds and 32-byte edge quads at random; a
// cache line is 128 bytes).
#include <hip/hip_runtime.h>

#include "skis_internal.h"

namespace skis {

// lowbias32 (C. Wellons, hash-prospector): a 32-bit mixing function good enough to spread
// read positions uniformly over the table
__device__ __forceinline__ uint32_t probe_mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// Row r of read i: floor(mix(i ^ seed') * rows / 2^32) < rows, so every read is in bounds.
__device__ __forceinline__ uint32_t probe_row(uint32_t i, uint32_t seed, uint32_t rows)
{
    return (uint32_t)(((uint64_t)probe_mix(i ^ seed) * rows) >> 32);
}

template <int ROWB>
__device__ __forceinline__ uint32_t probe_read(const unsigned char *table, uint32_t r)
{
    if constexpr (ROWB == 8) {
        const uint2 v = *reinterpret_cast<const uint2 *>(table + (size_t)r * 8);
        return v.x ^ v.y;
    } else {
        const uint4 *p = reinterpret_cast<const uint4 *>(table + (size_t)r * ROWB);
        uint32_t a = 0u;
#pragma unroll
        for (int k = 0; k < ROWB / 16; ++k) {
            const uint4 v = p[k];
            a ^= v.x ^ v.y ^ v.z ^ v.w;
        }
        return a;
    }
}

// Each thread takes reads i = gid, gid + stride, ...; four independent rows are in flight
// per thread and iteration.  The rows' words are folded into one value that is stored only
// if it equals a fixed constant, which keeps the loads without writing anything in practice.
// The read index is 64-bit, so the loop ends for every accepted count (reads < 2^32).
template <int ROWB>
__global__ __launch_bounds__(256) void k_probe_random_read(const unsigned char *table, uint32_t rows,
                                                           uint64_t reads, uint32_t seed, uint32_t *sink)
{
    constexpr uint64_t U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0u;
    for (; i + (U - 1) * stride < reads; i += U * stride) {
        uint32_t r[U], v[U];
#pragma unroll
        for (uint32_t k = 0; k < U; ++k) r[k] = probe_row((uint32_t)(i + k * stride), seed, rows);
#pragma unroll
        for (uint32_t k = 0; k < U; ++k) v[k] = probe_read<ROWB>(table, r[k]);
#pragma unroll
        for (uint32_t k = 0; k < U; ++k) acc ^= v[k];
    }
    for (; i < reads; i += stride) acc ^= probe_read<ROWB>(table, probe_row((uint32_t)i, seed, rows));
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

void probe_random_read(const void *table, uint64_t rows, uint32_t row_bytes, uint64_t reads, uint32_t seed,
                       uint32_t *sink, hipStream_t s)
{
    if (!table || !sink) throw Error{SKIS_EINVAL, "NULL argument"};
    if (rows == 0 || rows > 0xFFFFFFFFull) throw Error{SKIS_EINVAL, "rows must be in [1, 2^32)"};
    if (reads > 0xFFFFFFFFull) throw Error{SKIS_EINVAL, "reads must be below 2^32"};
    if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0) throw Error{SKIS_EINVAL, "table must be 16-byte aligned"};
    if (reads == 0) return;
    const unsigned grid = (unsigned)device_cu_count() * 16u;
    const uint32_t nr = (uint32_t)rows;
    const uint64_t nreads = reads;
    const unsigned char *t = static_cast<const unsigned char *>(table);
    switch (row_bytes) {
    case 8: hipLaunchKernelGGL(k_probe_random_read<8>, dim3(grid), dim3(256), 0, s, t, nr, nreads, seed, sink); break;
    case 16: hipLaunchKernelGGL(k_probe_random_read<16>, dim3(grid), dim3(256), 0, s, t, nr, nreads, seed, sink); break;
    case 32: hipLaunchKernelGGL(k_probe_random_read<32>, dim3(grid), dim3(256), 0, s, t, nr, nreads, seed, sink); break;
    case 64: hipLaunchKernelGGL(k_probe_random_read<64>, dim3(grid), dim3(256), 0, s, t, nr, nreads, seed, sink); break;
    case 128: hipLaunchKernelGGL(k_probe_random_read<128>, dim3(grid), dim3(256), 0, s, t, nr, nreads, seed, sink); break;
    default: throw Error{SKIS_EINVAL, "row_bytes must be 8, 16, 32, 64 or 128"};
    }
    SKIS_HIP_TRY(hipGetLastError());
}

} // namespace skis
