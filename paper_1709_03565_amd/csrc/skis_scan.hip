// skis_scan.hip -- device-wide exclusive prefix sums (three passes: tile reduce, scan of
// tile sums, tile scan with carry-in).  Integer types only, so the result does not depend
// on the order of additions.
#include "skis_internal.h"

namespace skis {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Exclusive scan of one value per thread across the block; LDS only, works for u128.
template <typename T>
__device__ T block_scan_lds(T v, T *sh, T *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    if (t < 64) {
        // each of the 64 lanes owns 4 consecutive entries
        T a0 = sh[4 * t], a1 = sh[4 * t + 1], a2 = sh[4 * t + 2], a3 = sh[4 * t + 3];
        T s = a0 + a1 + a2 + a3;
        T inc = s;
        for (int d = 1; d < 64; d <<= 1) {
            // shuffles of u128 are split into two 64-bit halves
            uint64_t lo = (uint64_t)inc, hi = (uint64_t)((u128)inc >> 64);
            uint64_t olo = __shfl_up(lo, d, 64), ohi = __shfl_up(hi, d, 64);
            T o = (T)(((u128)ohi << 64) | olo);
            if (t >= d) inc += o;
        }
        T ex = inc - s;
        sh[4 * t] = ex;
        sh[4 * t + 1] = ex + a0;
        sh[4 * t + 2] = ex + a0 + a1;
        sh[4 * t + 3] = ex + a0 + a1 + a2;
        if (t == 63) sh[SCAN_BLOCK] = inc;
    }
    __syncthreads();
    T r = sh[t];
    *total = sh[SCAN_BLOCK];
    __syncthreads();
    return r;
}

template <typename S, typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const S *in, int64_t n, T *partials)
{
    __shared__ T sh[SCAN_BLOCK + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + threadIdx.x + (int64_t)k * SCAN_BLOCK;
        if (i < n) acc += (T)in[i];
    }
    T total;
    block_scan_lds<T>(acc, sh, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(T *partials, int64_t nb, T *total_out)
{
    __shared__ T sh[SCAN_BLOCK + 1];
    T carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
        int64_t i = b0 + threadIdx.x;
        T v = i < nb ? partials[i] : (T)0;
        T tot;
        T ex = block_scan_lds<T>(v, sh, &tot);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename S, typename T, typename D>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(const S *in, D *out, int64_t n, const T *partials)
{
    __shared__ T tile[SCAN_TILE];
    __shared__ T sh[SCAN_BLOCK + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int idx = threadIdx.x + k * SCAN_BLOCK;
        int64_t i = base + idx;
        tile[idx] = i < n ? (T)in[i] : (T)0;
    }
    __syncthreads();
    T loc[SCAN_ITEMS];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        loc[k] = acc;
        acc += tile[threadIdx.x * SCAN_ITEMS + k];
    }
    T tot;
    T ex = block_scan_lds<T>(acc, sh, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) tile[threadIdx.x * SCAN_ITEMS + k] = ex + loc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int idx = threadIdx.x + k * SCAN_BLOCK;
        int64_t i = base + idx;
        if (i < n) out[i] = (D)tile[idx];
    }
}

template <typename S, typename T, typename D>
static void scan_impl(Arena &arena, const S *in, D *out, int64_t n, T *d_total, hipStream_t s)
{
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    DevBuf<T> part;
    part.alloc(arena, (size_t)(nb > 0 ? nb : 1));
    if (nb > 0) {
        hipLaunchKernelGGL((k_scan_reduce<S, T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, part.ptr);
        SKIS_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL((k_scan_tiles<T>), dim3(1), dim3(SCAN_BLOCK), 0, s, part.ptr, nb, d_total);
    SKIS_HIP_TRY(hipGetLastError());
    if (nb > 0) {
        hipLaunchKernelGGL((k_scan_down<S, T, D>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n,
                           part.ptr);
        SKIS_HIP_TRY(hipGetLastError());
    }
    // `part` is released on return, ordered on the arena's stream after the kernels above
    // (or by a synchronising free when the device has no memory pool).
}

template <typename T>
void excl_scan(Arena &arena, const T *in, T *out, int64_t n, T *d_total, hipStream_t s)
{
    scan_impl<T, T, T>(arena, in, out, n, d_total, s);
}

void excl_scan_u32_to_i64(Arena &arena, const uint32_t *in, int64_t *out, int64_t n, int64_t *d_total,
                          hipStream_t s)
{
    scan_impl<uint32_t, int64_t, int64_t>(arena, in, out, n, d_total, s);
}

template void excl_scan<uint32_t>(Arena &, const uint32_t *, uint32_t *, int64_t, uint32_t *, hipStream_t);
template void excl_scan<uint64_t>(Arena &, const uint64_t *, uint64_t *, int64_t, uint64_t *, hipStream_t);
template void excl_scan<int64_t>(Arena &, const int64_t *, int64_t *, int64_t, int64_t *, hipStream_t);
template void excl_scan<u128>(Arena &, const u128 *, u128 *, int64_t, u128 *, hipStream_t);

} // namespace skis
