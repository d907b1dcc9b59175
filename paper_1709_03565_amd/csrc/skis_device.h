// skis_device.h -- device helpers shared by the libskis HIP sources (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace skis {

typedef unsigned __int128 u128;

constexpr uint32_t TAG_ROOT = 0u;   // Philox tag: root draw
constexpr uint32_t TAG_FIRST = 1u;  // Philox tag: first live in-edge of the root
constexpr uint32_t TAG_EDGE = 2u;   // Philox tag: high halves of the live-edge coins, four edges per call
constexpr uint32_t TAG_EDGE_LOW = 3u; // Philox tag: low half of one edge's coin
constexpr uint32_t TAG_LT = 4u;    // Philox tag: the in-neighbour a node picks under the linear threshold model

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64-bit
// multiplications with Weyl-bumped keys.  Returns the two 64-bit halves X = y1:y0 and
// Y = y3:y2 of the output block for counter (c0, c1, c2, c3) and key (k0, k1).
__device__ __forceinline__ void philox2x64(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1, uint64_t &X, uint64_t &Y)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XORs in one gfx950 instruction each (truth table 0x96: odd parity)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    X = ((uint64_t)c1 << 32) | c0;
    Y = ((uint64_t)c3 << 32) | c2;
}

// floor(w * 2^64) for a non-negative float w < 1 given by its bits, in integer arithmetic:
// w = man * 2^(ex-150) for a normal number, so w * 2^64 = man * 2^(ex-86).
__device__ __forceinline__ uint64_t coin_threshold(uint32_t wbits)
{
    const uint32_t ex = wbits >> 23;
    if (ex == 0u) return 0ull; // zero or subnormal: below 2^-126, times 2^64 is < 1
    const uint64_t man = (uint64_t)((wbits & 0x7FFFFFu) | 0x800000u);
    if (ex >= 86u) return man << (ex - 86u);
    const uint32_t sh = 86u - ex;
    return sh >= 24u ? 0ull : (man >> sh);
}

// An edge of probability w (bits of a float in [0,1], +0 for zero) is live for a 64-bit
// uniform word x iff w >= 1 or x < floor(w * 2^64): probability exactly w for w >= 2^-40.
__device__ __forceinline__ bool coin_live(uint32_t wbits, uint64_t x)
{
    return wbits >= 0x3F800000u || x < coin_threshold(wbits);
}

// The high half of the coin threshold floor(w * 2^64), or 0xFFFFFFFF for w >= 1.  An edge
// whose coin has a high half below it is live, one above it is not, and one equal to it is
// decided by coin_live on the whole coin (for w < 1 the threshold's high half is at most
// 0xFFFFFF00, so 0xFFFFFFFF is free to mean "always live").
__device__ __forceinline__ uint32_t coin_threshold_hi(uint32_t wbits)
{
    return wbits >= 0x3F800000u ? 0xFFFFFFFFu : (uint32_t)(coin_threshold(wbits) >> 32);
}

// The whole 64-bit coin of edge e in sample j given its high half: the low half is word 0
// of the call with counter (e, j_lo, j_hi, TAG_EDGE_LOW).
__device__ __forceinline__ uint64_t coin_with_low_half(uint32_t hi, uint32_t e, uint64_t j, uint32_t seed_lo,
                                                       uint32_t seed_hi)
{
    uint64_t X, Y;
    philox2x64(e, (uint32_t)j, (uint32_t)(j >> 32), TAG_EDGE_LOW, seed_lo, seed_hi, X, Y);
    return ((uint64_t)hi << 32) | (uint32_t)X;
}

// Field at byte offset `off` of the kernel's argument segment, read with a scalar load at the
// point of use.  The empty asm hides the segment's address from the optimiser, so the load is
// not hoisted out of loops: an argument used once per pass or less then holds no scalar
// register across a persistent kernel's loop (where it would be spilled to a VGPR lane and
// reloaded with a VALU instruction at each use).
template <typename T>
__device__ __forceinline__ T karg_at(size_t off)
{
    const char __attribute__((address_space(4))) *base =
        (const char __attribute__((address_space(4))) *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(base));
    return *(const T __attribute__((address_space(4))) *)(base + off);
}

// Alias-table entry: bucket b yields b when r < thr, else alias.
struct __align__(16) AliasEntry {
    uint64_t thr;
    int32_t alias;
    int32_t pad;
};

// Adds lane (l - d) of the same row of 16 lanes to lane l (nothing where l mod 16 < d), d in
// {1, 2, 4, 8}: one DPP-modified VALU add, no LDS traffic.
template <int D>
__device__ __forceinline__ uint32_t dpp_row_shr_add(uint32_t x)
{
    return x + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + D, 0xf, 0xf, true);
}

// Inclusive prefix sum of 32-bit values over the 64 lanes by DPP: a scan within each row of 16
// (row_shr 1, 2, 4, 8), then lane 15 of rows 0 and 2 into rows 1 and 3 (row_bcast:15), then
// lane 31 into rows 2 and 3 (row_bcast:31).  Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x)
{
    x = dpp_row_shr_add<1>(x);
    x = dpp_row_shr_add<2>(x);
    x = dpp_row_shr_add<4>(x);
    x = dpp_row_shr_add<8>(x);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x;
}

// max(x, lane (l - d) of the same row of 16 lanes) in lane l (x where l mod 16 < d), d in
// {1, 2, 4, 8}.
template <int D>
__device__ __forceinline__ uint32_t dpp_row_shr_max(uint32_t x)
{
    const uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + D, 0xf, 0xf, true);
    return x > y ? x : y;
}

// Inclusive prefix maximum over the 64 lanes (unsigned; every lane active): the same steps
// as wave_incl_scan_dpp with max for +.
__device__ __forceinline__ uint32_t wave_incl_max_dpp(uint32_t x)
{
    x = dpp_row_shr_max<1>(x);
    x = dpp_row_shr_max<2>(x);
    x = dpp_row_shr_max<4>(x);
    x = dpp_row_shr_max<8>(x);
    uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x > y ? x : y;
}

// Wave-level inclusive prefix sum over the 64 lanes (every lane active).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    if constexpr (sizeof(T) == 4) {
        return (T)wave_incl_scan_dpp((uint32_t)v);
    } else {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T o = __shfl_up(v, d, 64);
            if (lane >= d) v += o;
        }
        return v;
    }
}

// Value of lane `lane` (a constant) / of the first active lane, through a scalar register
// (no LDS traffic, unlike a shuffle).
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ unsigned long long lane_value64(unsigned long long v, int lane)
{
    const uint32_t lo = lane_value((uint32_t)v, lane), hi = lane_value((uint32_t)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long first_lane_value64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Inclusive prefix sum over lanes 0 .. N-1 (exact there; lanes from N on hold partial sums),
// 32-bit values, every lane active.
template <int N, typename T>
__device__ __forceinline__ T wave_incl_scan_n(T v)
{
    static_assert(sizeof(T) == 4, "32-bit scan");
    if constexpr (N > 16) {
        return (T)wave_incl_scan_dpp((uint32_t)v);
    } else {
        uint32_t x = (uint32_t)v;
        if constexpr (N > 1) x = dpp_row_shr_add<1>(x);
        if constexpr (N > 2) x = dpp_row_shr_add<2>(x);
        if constexpr (N > 4) x = dpp_row_shr_add<4>(x);
        if constexpr (N > 8) x = dpp_row_shr_add<8>(x);
        return (T)x;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Workgroup barrier.  A one-wave workgroup only needs its LDS operations ordered: the
// wavefront-scope fences keep the compiler from moving LDS accesses across the call and
// the wave issues its LDS instructions in order, so no wait for outstanding global memory
// operations is forced (s_barrier with a full waitcnt would be).
template <int BLOCK>
__device__ __forceinline__ void block_sync()
{
    if constexpr (BLOCK == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Block exclusive prefix sum of one value per thread.  `ws` is LDS scratch of at least
// BLOCK/64 + 1 entries; for more than one wave the call contains two barriers.  Returns
// the block total in *total.  Every thread of the block must call it.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *ws, T *total)
{
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if constexpr (NW == 1) {
        (void)ws;
        *total = __shfl(inc, 63, 64);
        return inc - v;
    }
    if (lane == 63) ws[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < NW; ++i) {
            T t = ws[i];
            ws[i] = acc;
            acc += t;
        }
        ws[NW] = acc;
    }
    __syncthreads();
    *total = ws[NW];
    return ws[wid] + inc - v;
}

// Round-to-nearest-even conversion of an unsigned 128-bit integer to binary64.
__device__ __forceinline__ double u128_to_double(u128 x)
{
    if (x == 0) return 0.0;
    const uint64_t hi = (uint64_t)(x >> 64);
    const int lz = hi ? __clzll((long long)hi) : 64 + __clzll((long long)(uint64_t)x);
    const int msb = 127 - lz;
    if (msb <= 52) return (double)(uint64_t)x; // exact
    const int sh = msb - 52;
    uint64_t mant = (uint64_t)(x >> sh);
    const u128 rem = x & (((u128)1 << sh) - 1);
    const u128 half = (u128)1 << (sh - 1);
    int e = sh;
    if (rem > half || (rem == half && (mant & 1ull))) {
        ++mant;
        if (mant == (1ull << 53)) {
            mant >>= 1;
            ++e;
        }
    }
    return ldexp((double)mant, e);
}

} // namespace skis
