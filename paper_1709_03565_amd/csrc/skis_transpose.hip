// skis_transpose.hip -- node -> samples transpose of the sketch by a stable LSD radix sort of
// the (node, sample) pairs on the node id, 8 bits per pass.
//
// A direct scatter from the sketch writes one 4-byte id per entry to a random place in HBM
// (each write a partial-line update).  The sort instead writes every pass in runs: each
// tile of RS_TILE entries sends its entries of one digit to one contiguous range.  Per pass:
//   k_rs_hist     digit counts per tile, one contiguous row per tile; per-chunk digit sums,
//                 one exclusive scan of those (digit-major) and a walk over each chunk's rows
//                 give every (tile, digit) its output offset, again one row per tile;
//   k_rs_scatter  each wave ranks its entries among equal digits with one ballot per digit
//                 bit (lanes in order) in one pass that also counts the wave's digits, the
//                 waves of a tile are ordered by a prefix of their counts, the tile is sorted
//                 by digit in LDS (stable) and written out in order, so each digit's run of
//                 the tile goes to its offset with consecutive lanes.
// The input is in sample order, so every list H(v) comes out sorted by sample id.
// The last pass writes only the sample ids and counts each node's entries; node_ptr is the
// exclusive scan of those counts.
#include <algorithm>

#include "skis_internal.h"

namespace skis {

constexpr int RS_BLOCK = 1024;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_TILE = 16384;                // entries per tile (digit runs of ~64 entries)
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
        if (threadIdx.x < 256) h[threadIdx.x] = 0u;
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
        if (threadIdx.x < 256) H[tile * 256 + threadIdx.x] = h[threadIdx.x]; // one contiguous row per tile
        __syncthreads();
    }
}

// Output offsets of every (tile, digit) from the tile-major histogram H[tile][digit]: the
// entries of digit d go after those of every smaller digit and, within d, tile by tile.
// k_rs_chunk_sums adds the rows of each chunk of RS_CHUNK tiles per digit into C[d][chunk]
// (digit-major, so one exclusive scan of C gives every (digit, chunk) its base), and
// k_rs_offsets walks the chunk's rows from that base, writing OFF[tile][digit].  Every access
// to H and OFF is a contiguous row of 256 values.
constexpr int RS_CHUNK = 64;

__global__ __launch_bounds__(256) void k_rs_chunk_sums(uint64_t ntiles, const uint32_t *__restrict__ H,
                                                       uint64_t nchunks, uint32_t *__restrict__ C)
{
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t t0 = c * RS_CHUNK, t1 = min(t0 + RS_CHUNK, ntiles);
        uint32_t acc = 0;
        for (uint64_t t = t0; t < t1; ++t) acc += H[t * 256 + threadIdx.x];
        C[(uint64_t)threadIdx.x * nchunks + c] = acc;
    }
}

__global__ __launch_bounds__(256) void k_rs_offsets(uint64_t ntiles, const uint32_t *__restrict__ H,
                                                    uint64_t nchunks, const int64_t *__restrict__ CB,
                                                    int64_t *__restrict__ OFF)
{
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t t0 = c * RS_CHUNK, t1 = min(t0 + RS_CHUNK, ntiles);
        int64_t acc = CB[(uint64_t)threadIdx.x * nchunks + c];
        for (uint64_t t = t0; t < t1; ++t) {
            OFF[t * 256 + threadIdx.x] = acc;
            acc += H[t * 256 + threadIdx.x];
        }
    }
}

// Lanes of the wave holding the same digit d as this lane (among the valid ones); digits
// have `bits` significant bits (uniform), the others are zero.
__device__ __forceinline__ unsigned long long same_digit_mask(bool valid, uint32_t d, int bits)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (b >= bits) break;
        const bool bit = (d >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(RS_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_rs_scatter(uint64_t N, const int32_t *__restrict__ kin,
                                                         const int32_t *__restrict__ vin, int32_t *__restrict__ kout,
                                                         int32_t *__restrict__ vout, int shift, int bits,
                                                         uint64_t ntiles, const int64_t *__restrict__ OFF,
                                                         uint32_t *__restrict__ deg)
{
    __shared__ long long base[256];        // output offset of each digit for this tile
    __shared__ uint32_t tstart[256 + 1];   // first tile-local position of each digit
    __shared__ uint32_t cnt[RS_WAVES][256]; // per-wave digit counts, then each wave's running index
    __shared__ int32_t sk[RS_TILE], sv[RS_TILE]; // the tile, then the tile sorted by digit
    __shared__ uint32_t s_scan[RS_WAVES + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    constexpr int R = RS_SPAN / 64;
    constexpr int PER = RS_TILE / RS_BLOCK;
    // the next tile's entries and digit offsets are loaded while this one is sorted and
    // written (unconditional loads: an index past the end reads the last entry, unused)
    int32_t kr[R], vr[R];
    long long bnext = 0;
    uint64_t tile = blockIdx.x;
    if (tile < ntiles) {
        const uint64_t s0 = tile * RS_TILE + (uint64_t)w * RS_SPAN;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t e = min(s0 + (uint64_t)r * 64 + lane, N - 1);
            kr[r] = kin[e];
            vr[r] = vin[e];
        }
        if (threadIdx.x < 256) bnext = OFF[tile * 256 + threadIdx.x];
    }
    for (; tile < ntiles; tile += gridDim.x) {
        const uint64_t t0 = tile * RS_TILE;
        const uint64_t s0 = t0 + (uint64_t)w * RS_SPAN;
        const int nvalid = (int)min((uint64_t)RS_TILE, N - t0);
        if (threadIdx.x < 256) base[threadIdx.x] = bnext;
        for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_BLOCK) (&cnt[0][0])[i] = 0u;
        const uint64_t tn = tile + gridDim.x;
        if (tn < ntiles && threadIdx.x < 256) bnext = OFF[tn * 256 + threadIdx.x];
        __syncthreads();
        // one ranking pass over the wave's span (in registers, in order): the rank of each
        // entry among the equal digits before it in the wave, while the leader of each digit
        // and round advances the wave's count of that digit
        uint32_t lp[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool valid = s0 + (uint64_t)r * 64 + lane < N;
            const uint32_t d = valid ? (((uint32_t)kr[r] >> shift) & 255u) : 0u;
            const unsigned long long m = same_digit_mask(valid, d, bits);
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
        // digit d of the tile: its waves in order, after the digits below d
        {
            const int d = threadIdx.x; // digits 0..255; the other threads add nothing
            uint32_t acc = 0;
            if (d < 256)
                for (int k = 0; k < RS_WAVES; ++k) {
                    const uint32_t x = cnt[k][d];
                    cnt[k][d] = acc;
                    acc += x;
                }
            uint32_t tot;
            const uint32_t ex = block_excl_scan<RS_BLOCK, uint32_t>(acc, s_scan, &tot);
            if (d < 256) {
                tstart[d] = ex;
                if (d == 255) tstart[256] = tot;
                for (int k = 0; k < RS_WAVES; ++k) cnt[k][d] += ex;
            }
        }
        __syncthreads();
        // the tile sorted by digit (stably) in LDS
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (lp[r] != 0xFFFFFFFFu) {
                const uint32_t d = ((uint32_t)kr[r] >> shift) & 255u;
                const uint32_t pos = cnt[w][d] + lp[r];
                sk[pos] = kr[r];
                sv[pos] = vr[r];
            }
        __syncthreads();
        // the next tile's loads go out before this one is written
        if (tn < ntiles) {
            const uint64_t n0 = tn * RS_TILE + (uint64_t)w * RS_SPAN;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t e = min(n0 + (uint64_t)r * 64 + lane, N - 1);
                kr[r] = kin[e];
                vr[r] = vin[e];
            }
        }
        // phase 3: the sorted tile goes out in order, each digit's run to its offset.  In the
        // last pass (deg set) the keys are not written: each run of equal keys within a
        // digit's run adds its length to deg[key], as -first at its first element and
        // last + 1 at its last one (the pass's keys are sorted within a digit's run).
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * RS_BLOCK + threadIdx.x;
            if (i < nvalid) {
                const int32_t key = sk[i];
                const uint32_t d = ((uint32_t)key >> shift) & 255u;
                const long long pos = base[d] + (long long)(i - (int)tstart[d]);
                vout[pos] = sv[i];
                if (!deg) {
                    kout[pos] = key;
                } else {
                    const bool first = i == (int)tstart[d] || sk[i - 1] != key;
                    const bool last = i + 1 == (int)tstart[d + 1] || sk[i + 1] != key;
                    if (first) atomicAdd(&deg[key], (uint32_t)(-i));
                    if (last) atomicAdd(&deg[key], (uint32_t)(i + 1));
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rs_fill_u32(uint64_t count, uint32_t *__restrict__ p, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_rs(uint64_t items, int block, int per_cu = 8)
{
    uint64_t g = (items + block - 1) / block;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

void radix_transpose(Arena &arena, const int64_t *sample_ptr, const int32_t *nodes, int32_t *owner, uint64_t T,
                     uint64_t N, int32_t n, int64_t *node_ptr, int32_t *node_samples, uint32_t *deg, hipStream_t s)
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
    int32_t *vals = owner; // the sample id of every entry, scratch after the first pass
    if (!vals) {
        va.alloc(arena, N);
        vals = va.ptr;
    }
    if (passes > 1) vb.alloc(arena, N);
    kb.alloc(arena, N);
    const uint64_t nchunks = (ntiles + RS_CHUNK - 1) / RS_CHUNK;
    H.alloc(arena, 256 * ntiles);
    OFF.alloc(arena, 256 * ntiles);
    DevBuf<uint32_t> C;
    DevBuf<int64_t> CB;
    C.alloc(arena, 256 * nchunks);
    CB.alloc(arena, 256 * nchunks + 1);
    if (!owner) {
        hipLaunchKernelGGL(k_rs_vals, dim3(grid_rs(T * 64, 256, 16)), dim3(256), 0, s, T, sample_ptr, vals);
        SKIS_HIP_TRY(hipGetLastError());
    }
    const unsigned gt = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)device_cu_count() * 8);
    // pass p reads (kin, vin) and writes (kout, vout); the sketch's nodes are the first keys,
    // the last pass writes the values straight into node_samples
    const int32_t *kin = nodes;
    const int32_t *vin = vals;
    // the last pass counts each node's entries instead of writing the sorted keys
    hipLaunchKernelGGL(k_rs_fill_u32, dim3(grid_rs(n, 256, 4)), dim3(256), 0, s, (uint64_t)n, deg, 0u);
    for (int p = 0; p < passes; ++p) {
        const bool lastp = p == passes - 1;
        int32_t *kout = lastp ? nullptr : ((p & 1) ? ka.ptr : kb.ptr);
        int32_t *vout = lastp ? node_samples : ((p & 1) ? vals : vb.ptr);
        hipLaunchKernelGGL(k_rs_hist, dim3(gt), dim3(RS_BLOCK), 0, s, N, kin, 8 * p, ntiles, H.ptr);
        SKIS_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_rs_chunk_sums, dim3(grid_rs(nchunks * 256, 256, 8)), dim3(256), 0, s, ntiles, H.ptr,
                           nchunks, C.ptr);
        excl_scan_u32_to_i64(arena, C.ptr, CB.ptr, (int64_t)(256 * nchunks), CB.ptr + 256 * nchunks, s);
        hipLaunchKernelGGL(k_rs_offsets, dim3(grid_rs(nchunks * 256, 256, 8)), dim3(256), 0, s, ntiles, H.ptr,
                           nchunks, CB.ptr, OFF.ptr);
        SKIS_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_rs_scatter, dim3(gt), dim3(RS_BLOCK), 0, s, N, kin, vin, kout, vout, 8 * p,
                           std::min(8, bits - 8 * p), ntiles, OFF.ptr, lastp ? deg : nullptr);
        SKIS_HIP_TRY(hipGetLastError());
        kin = kout;
        vin = vout;
    }
    excl_scan_u32_to_i64(arena, deg, node_ptr, n, node_ptr + n, s);
    SKIS_HIP_TRY(hipStreamSynchronize(s)); // the temporaries are released on return
}

} // namespace skis
