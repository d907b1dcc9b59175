// skis_transpose.hip -- node -> samples transpose of the sketch by a stable LSD radix sort of
// the (node, sample) pairs on the node id, 8 bits per pass.
//
// A direct scatter from the sketch writes one 4-byte id per entry to a random place in HBM
// (each write a partial-line update).  The sort instead writes every pass in runs: each
// tile of RS_TILE entries sends its entries of one digit to one contiguous range.  Per pass:
//   k_rs_hist     digit counts per tile, stored digit-major (H[d * ntiles + tile]), so one
//                 exclusive scan of H gives every (tile, digit) its output offset;
//   k_rs_scatter  each wave ranks its entries among equal digits with 8 ballots (lanes in
//                 order), the waves of a tile are ordered by a prefix of their counts, the
//                 tile is sorted by digit in LDS (stable) and written out in order, so each
//                 digit's run of the tile goes to its offset with consecutive lanes.
// The input is in sample order, so every list H(v) comes out sorted by sample id.
// k_rs_bounds then finds where each node's run starts.
#include <algorithm>

#include "skis_internal.h"

namespace skis {

constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_TILE = 4096;                 // entries per tile
constexpr int RS_SPAN = RS_TILE / RS_WAVES;   // entries per wave, in rounds of 64

// vals[p] = j for every entry p of sample j (one wave per sample)
__global__ __launch_bounds__(256) void k_rs_vals(uint64_t T, const int64_t *__restrict__ sptr,
                                                 int32_t *__restrict__ vals)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t j = wid; j < T; j += nw) {
        const int64_t a = sptr[j], b = sptr[j + 1];
        for (int64_t p = a + lane; p < b; p += 64) vals[p] = (int32_t)j;
    }
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(uint64_t N, const int32_t *__restrict__ keys, int shift,
                                                      uint64_t ntiles, uint32_t *__restrict__ H)
{
    __shared__ uint32_t h[256];
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        h[threadIdx.x] = 0u;
        __syncthreads();
        const uint64_t e0 = tile * RS_TILE;
        constexpr int R = RS_TILE / RS_BLOCK;
        int32_t kr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t e = e0 + (uint64_t)r * RS_BLOCK + threadIdx.x;
            kr[r] = e < N ? keys[e] : -1;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (kr[r] >= 0) atomicAdd(&h[((uint32_t)kr[r] >> shift) & 255u], 1u);
        __syncthreads();
        H[(uint64_t)threadIdx.x * ntiles + tile] = h[threadIdx.x];
        __syncthreads();
    }
}

// Lanes of the wave holding the same digit d as this lane (among the valid ones).
__device__ __forceinline__ unsigned long long same_digit_mask(bool valid, uint32_t d)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(uint64_t N, const int32_t *__restrict__ kin,
                                                         const int32_t *__restrict__ vin, int32_t *__restrict__ kout,
                                                         int32_t *__restrict__ vout, int shift, uint64_t ntiles,
                                                         const int64_t *__restrict__ OFF)
{
    __shared__ long long base[256];        // output offset of each digit for this tile
    __shared__ uint32_t tstart[256 + 1];   // first tile-local position of each digit
    __shared__ uint32_t cnt[RS_WAVES][256]; // per-wave digit counts, then each wave's running index
    __shared__ int32_t sk[RS_TILE], sv[RS_TILE]; // the tile, then the tile sorted by digit
    __shared__ uint32_t s_scan[RS_WAVES + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    constexpr int R = RS_SPAN / 64;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        base[threadIdx.x] = OFF[(uint64_t)threadIdx.x * ntiles + tile];
        for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_BLOCK) (&cnt[0][0])[i] = 0u;
        const uint64_t t0 = tile * RS_TILE;
        const uint64_t s0 = t0 + (uint64_t)w * RS_SPAN;
        const int nvalid = (int)min((uint64_t)RS_TILE, N - t0);
        {
            // the wave's span: all loads in flight at once, then staged in LDS
            int32_t kr[R], vr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t e = s0 + (uint64_t)r * 64 + lane;
                kr[r] = e < N ? kin[e] : 0;
                vr[r] = e < N ? vin[e] : 0;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sk[w * RS_SPAN + r * 64 + lane] = kr[r];
                sv[w * RS_SPAN + r * 64 + lane] = vr[r];
            }
        }
        __syncthreads();
        // phase 1: this wave's digit counts (one leader per digit and round adds)
        for (int r = 0; r < R; ++r) {
            const bool valid = s0 + (uint64_t)r * 64 + lane < N;
            const uint32_t d = valid ? (((uint32_t)sk[w * RS_SPAN + r * 64 + lane] >> shift) & 255u) : 0u;
            const unsigned long long m = same_digit_mask(valid, d);
            if (valid && !(m & lt)) cnt[w][d] += (uint32_t)__popcll(m);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        // digit d of the tile: its waves in order, after the digits below d
        {
            const int d = threadIdx.x;
            uint32_t acc = 0;
            for (int k = 0; k < RS_WAVES; ++k) {
                const uint32_t x = cnt[k][d];
                cnt[k][d] = acc;
                acc += x;
            }
            uint32_t tot;
            const uint32_t ex = block_excl_scan<RS_BLOCK, uint32_t>(acc, s_scan, &tot);
            tstart[d] = ex;
            if (d == 255) tstart[256] = tot;
            for (int k = 0; k < RS_WAVES; ++k) cnt[k][d] += ex;
        }
        __syncthreads();
        // phase 2: tile-local positions (stable), kept in registers until every wave has read
        int32_t kr[R], vr[R];
        uint32_t lp[R];
        for (int r = 0; r < R; ++r) {
            const bool valid = s0 + (uint64_t)r * 64 + lane < N;
            kr[r] = sk[w * RS_SPAN + r * 64 + lane];
            vr[r] = sv[w * RS_SPAN + r * 64 + lane];
            const uint32_t d = valid ? (((uint32_t)kr[r] >> shift) & 255u) : 0u;
            const unsigned long long m = same_digit_mask(valid, d);
            lp[r] = valid ? cnt[w][d] + (uint32_t)__popcll(m & lt) : 0xFFFFFFFFu;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid && !(m & lt)) cnt[w][d] += (uint32_t)__popcll(m);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        for (int r = 0; r < R; ++r)
            if (lp[r] != 0xFFFFFFFFu) {
                sk[lp[r]] = kr[r];
                sv[lp[r]] = vr[r];
            }
        __syncthreads();
        // phase 3: the sorted tile goes out in order, each digit's run to its offset
        for (int i = threadIdx.x; i < nvalid; i += RS_BLOCK) {
            const int32_t key = sk[i];
            const uint32_t d = ((uint32_t)key >> shift) & 255u;
            const long long pos = base[d] + (long long)(i - (int)tstart[d]);
            kout[pos] = key;
            vout[pos] = sv[i];
        }
        __syncthreads();
    }
}

// node_ptr[v] = first position of key v in the sorted keys (N past the last), for all v.
__global__ __launch_bounds__(256) void k_rs_bounds(uint64_t N, int32_t n, const int32_t *__restrict__ keys,
                                                   int64_t *__restrict__ node_ptr)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= N; p += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t prev = p > 0 ? keys[p - 1] : -1;
        const int32_t cur = p < N ? keys[p] : n;
        for (int32_t v = prev + 1; v <= cur && v <= n; ++v) node_ptr[v] = (int64_t)p;
    }
}

static unsigned grid_rs(uint64_t items, int block, int per_cu = 8)
{
    uint64_t g = (items + block - 1) / block;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

void radix_transpose(Arena &arena, const int64_t *sample_ptr, const int32_t *nodes, uint64_t T, uint64_t N,
                     int32_t n, int64_t *node_ptr, int32_t *node_samples, hipStream_t s)
{
    if (N == 0 || T == 0) throw Error{SKIS_EHIP, "internal error: empty transpose"};
    int bits = 1;
    while (bits < 31 && ((uint64_t)(n - 1) >> bits) != 0) ++bits;
    const int passes = (bits + 7) / 8;
    const uint64_t ntiles = (N + RS_TILE - 1) / RS_TILE;
    DevBuf<int32_t> ka, kb, va, vb;
    DevBuf<uint32_t> H;
    DevBuf<int64_t> OFF;
    ka.alloc(arena, N);
    va.alloc(arena, N);
    if (passes > 1) vb.alloc(arena, N);
    kb.alloc(arena, N);
    H.alloc(arena, 256 * ntiles);
    OFF.alloc(arena, 256 * ntiles + 1);
    hipLaunchKernelGGL(k_rs_vals, dim3(grid_rs(T * 64, 256, 16)), dim3(256), 0, s, T, sample_ptr, va.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    const unsigned gt = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)device_cu_count() * 8);
    // pass p reads (kin, vin) and writes (kout, vout); the sketch's nodes are the first keys,
    // the last pass writes the values straight into node_samples
    const int32_t *kin = nodes;
    const int32_t *vin = va.ptr;
    for (int p = 0; p < passes; ++p) {
        int32_t *kout = (p & 1) ? ka.ptr : kb.ptr;
        int32_t *vout = (p == passes - 1) ? node_samples : ((p & 1) ? va.ptr : vb.ptr);
        hipLaunchKernelGGL(k_rs_hist, dim3(gt), dim3(RS_BLOCK), 0, s, N, kin, 8 * p, ntiles, H.ptr);
        SKIS_HIP_TRY(hipGetLastError());
        excl_scan_u32_to_i64(arena, H.ptr, OFF.ptr, (int64_t)(256 * ntiles), OFF.ptr + 256 * ntiles, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(gt), dim3(RS_BLOCK), 0, s, N, kin, vin, kout, vout, 8 * p, ntiles,
                           OFF.ptr);
        SKIS_HIP_TRY(hipGetLastError());
        kin = kout;
        vin = vout;
    }
    hipLaunchKernelGGL(k_rs_bounds, dim3(grid_rs(N + 1, 256, 16)), dim3(256), 0, s, N, n, kin, node_ptr);
    SKIS_HIP_TRY(hipGetLastError());
    SKIS_HIP_TRY(hipStreamSynchronize(s)); // the temporaries are released on return
}

} // namespace skis
