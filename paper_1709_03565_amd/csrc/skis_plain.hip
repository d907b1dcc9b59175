// skis_plain.hip -- the plain form of the sampler: the reverse BFS of Alg. 1 advanced one
// level per launch over every sample of a chunk at once.  Visited sets live in one global
// open-addressing hash keyed by (sample, node); each level's frontier is a list of
// (sample, edge range) items whose edges are swept four at a time with the same Philox
// coins as the persistent sampler, so both forms produce the same sets.  The host reads
// the frontier size after every level.
#include <algorithm>

#include "skis_internal.h"
#include "skis_plain.h"

namespace skis {

constexpr unsigned long long HASH_EMPTY = ~0ull;
constexpr int PLAIN_BLOCK = 256;
constexpr int PLAIN_PPT = 4;                              // edge quads per thread per launch window
constexpr int PLAIN_WINDOW = PLAIN_BLOCK * PLAIN_PPT;     // quads per workgroup window
constexpr uint64_t PLAIN_MAX_PROBE = 4096;                // longest probe run before a resize

struct PlainCtx {
    const int32_t *row_ptr;
    const uint4 *pairs;              // edge records two at a time, padded to whole quads
    int64_t nquads;
    const uint32_t *wbits;           // w bits per edge: coin ties
    unsigned long long *hash;
    uint64_t hmask;
    uint32_t *sizes;                 // per sample of the chunk
    unsigned long long *probed;      // per sample of the chunk
    uint2 *entries;                  // (sample in chunk, node)
    unsigned long long *n_entries;
    uint64_t entries_cap;
    int4 *items_out;                 // (sample in chunk, edge begin, edge end, quads)
    unsigned long long *n_items_out;
    uint64_t items_cap;
    int *err;
};

__device__ __forceinline__ uint32_t quad_count(int32_t beg, int32_t end)
{
    return end > beg ? (uint32_t)(((end - 1) >> 2) - (beg >> 2) + 1) : 0u;
}

// Inserts (i, u); on success appends the entry and a frontier item for u's row.
__device__ __forceinline__ void plain_visit(const PlainCtx &c, uint32_t i, int32_t u)
{
    const unsigned long long key = ((unsigned long long)i << 32) | (uint32_t)u;
    uint64_t h = (key * 0x9E3779B97F4A7C15ull) >> 20;
    for (uint64_t probe = 0; probe < PLAIN_MAX_PROBE; ++probe) {
        h &= c.hmask;
        const unsigned long long old = atomicCAS(&c.hash[h], HASH_EMPTY, key);
        if (old == HASH_EMPTY) {
            atomicAdd(&c.sizes[i], 1u);
            const unsigned long long e = atomicAdd(c.n_entries, 1ull);
            if (e < c.entries_cap) c.entries[e] = make_uint2(i, (uint32_t)u);
            else atomicOr(c.err, 1);
            const int32_t rb = c.row_ptr[u], re = c.row_ptr[u + 1];
            atomicAdd(&c.probed[i], (unsigned long long)(re - rb));
            const uint32_t np = quad_count(rb, re);
            if (np) {
                const unsigned long long k = atomicAdd(c.n_items_out, 1ull);
                if (k < c.items_cap) c.items_out[k] = make_int4((int32_t)i, rb, re, (int32_t)np);
                else atomicOr(c.err, 2);
            }
            return;
        }
        if (old == key) return;
        ++h;
    }
    atomicOr(c.err, 4); // probe run too long: the chunk is redone with a larger table
}

// Level 0: root and first live in-edge of every sample; the root's later in-edges and the
// first neighbour's row form the first frontier.
__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_init(uint32_t count, uint32_t i0, const int4 *__restrict__ rec,
                                                            const int32_t *__restrict__ u1, PlainCtx c)
{
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const int4 r = rec[i0 + t];
        c.sizes[t] = 0u;
        c.probed[t] = (unsigned long long)(r.w - r.z);
        // the root: in R, its row handled by the root item below
        {
            const unsigned long long key = ((unsigned long long)t << 32) | (uint32_t)r.x;
            uint64_t h = (key * 0x9E3779B97F4A7C15ull) >> 20;
            bool done = false;
            for (uint64_t probe = 0; probe < PLAIN_MAX_PROBE && !done; ++probe) {
                h &= c.hmask;
                const unsigned long long old = atomicCAS(&c.hash[h], HASH_EMPTY, key);
                if (old == HASH_EMPTY || old == key) done = true;
                ++h;
            }
            if (!done) atomicOr(c.err, 4);
            atomicAdd(&c.sizes[t], 1u);
            const unsigned long long e = atomicAdd(c.n_entries, 1ull);
            if (e < c.entries_cap) c.entries[e] = make_uint2(t, (uint32_t)r.x);
            else atomicOr(c.err, 1);
        }
        const uint32_t np = quad_count(r.y + 1, r.w);
        if (np) {
            const unsigned long long k = atomicAdd(c.n_items_out, 1ull);
            if (k < c.items_cap) c.items_out[k] = make_int4((int32_t)t, r.y + 1, r.w, (int32_t)np);
            else atomicOr(c.err, 2);
        }
        const int32_t u = u1[i0 + t];
        if (u >= 0) plain_visit(c, t, u); // -1: a RIS sample, no first live in-edge
    }
}

__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_quads(uint64_t n_items, const int4 *__restrict__ items,
                                                             uint32_t *__restrict__ np)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_items; k += (uint64_t)gridDim.x * blockDim.x)
        np[k] = (uint32_t)items[k].w;
}

// One level: every edge quad of every frontier item.  Workgroup b takes quads
// [b*W, (b+1)*W); the items it touches are found once and their quad offsets staged in LDS.
__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_expand(uint64_t n_items, const int4 *__restrict__ items,
                                                              const int64_t *__restrict__ pbase, int64_t total,
                                                              uint32_t seed_lo, uint32_t seed_hi, uint64_t j0,
                                                              PlainCtx c)
{
    __shared__ int64_t s_pb[PLAIN_WINDOW + 2];
    __shared__ int64_t s_first;
    __shared__ int s_cnt;
    for (int64_t w0 = (int64_t)blockIdx.x * PLAIN_WINDOW; w0 < total; w0 += (int64_t)gridDim.x * PLAIN_WINDOW) {
        if (threadIdx.x == 0) { // last item whose first quad is <= w0
            int64_t lo = 0, hi = (int64_t)n_items - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (pbase[mid] <= w0) lo = mid; else hi = mid - 1;
            }
            s_first = lo;
            const int64_t rem = (int64_t)n_items - lo;
            s_cnt = (int)std::min<int64_t>(rem, PLAIN_WINDOW + 1);
        }
        __syncthreads();
        const int64_t first = s_first;
        const int cnt = s_cnt;
        for (int t = threadIdx.x; t < cnt; t += PLAIN_BLOCK) s_pb[t] = pbase[first + t];
        if (threadIdx.x == 0) s_pb[cnt] = first + cnt < (int64_t)n_items ? pbase[first + cnt] : total;
        __syncthreads();
        for (int g = 0; g < PLAIN_PPT; ++g) {
            const int64_t idx = w0 + (int64_t)g * PLAIN_BLOCK + threadIdx.x;
            if (idx >= total) break;
            int lo = 0, hi = cnt - 1; // last window item whose first quad is <= idx
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pb[mid] <= idx) lo = mid; else hi = mid - 1;
            }
            const int4 it = items[first + lo];
            const int qd = (it.y >> 2) + (int)(idx - s_pb[lo]);
            if (qd < 0 || (int64_t)qd >= c.nquads) { // bounds guard: report, never index
                atomicOr(c.err, 8);
                continue;
            }
            const uint4 p0 = c.pairs[2 * qd], p1 = c.pairs[2 * qd + 1];
            const uint32_t col[4] = {p0.x, p0.z, p1.x, p1.z}, th[4] = {p0.y, p0.w, p1.y, p1.w};
            const uint64_t j = j0 + (uint32_t)it.x;
            uint64_t X, Y;
            philox2x64((uint32_t)qd, (uint32_t)j, (uint32_t)(j >> 32), TAG_EDGE, seed_lo, seed_hi, X, Y);
            const uint32_t hw[4] = {(uint32_t)X, (uint32_t)(X >> 32), (uint32_t)Y, (uint32_t)(Y >> 32)};
            for (int h = 0; h < 4; ++h) {
                const int e = 4 * qd + h;
                if (e < it.y || e >= it.z) continue;
                const bool live = hw[h] != th[h]
                                      ? hw[h] < th[h]
                                      : coin_live(c.wbits[e], coin_with_low_half(hw[h], (uint32_t)e, j, seed_lo, seed_hi));
                if (live) plain_visit(c, (uint32_t)it.x, (int32_t)col[h]);
            }
        }
        __syncthreads();
    }
}

// Chunk compaction: entries into staging at the chunk's offsets (order within a sample is
// fixed later by the sort in the gather kernels).
__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_scatter(uint64_t n_entries, const uint2 *__restrict__ entries,
                                                               const int64_t *__restrict__ off, int64_t base,
                                                               uint32_t *__restrict__ fill, int32_t *__restrict__ staging,
                                                               uint64_t stage_cap, int *err)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_entries; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 e = entries[k];
        const int64_t pos = base + off[e.x] + (int64_t)atomicAdd(&fill[e.x], 1u);
        if ((uint64_t)pos < stage_cap) staging[pos] = (int32_t)e.y;
        else atomicOr(err, 16);
    }
}

__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_meta(uint32_t count, uint32_t i0, const uint32_t *__restrict__ sizes,
                                                            const unsigned long long *__restrict__ probed,
                                                            const int64_t *__restrict__ off, int64_t base,
                                                            uint32_t *__restrict__ out_size,
                                                            unsigned long long *__restrict__ out_off,
                                                            unsigned long long *__restrict__ out_probed,
                                                            uint32_t *__restrict__ medium,
                                                            unsigned long long *__restrict__ n_medium, int small_sort)
{
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const uint32_t i = i0 + t;
        out_size[i] = sizes[t];
        out_off[i] = (unsigned long long)(base + off[t]);
        out_probed[i] = probed[t];
        if ((int)sizes[t] > small_sort) medium[atomicAdd(n_medium, 1ull)] = i;
    }
}

template <typename T>
__global__ __launch_bounds__(PLAIN_BLOCK) void k_plain_fill(uint64_t count, T *__restrict__ p, T v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned gridp(uint64_t items, int per_cu = 16)
{
    uint64_t g = (items + PLAIN_BLOCK - 1) / PLAIN_BLOCK;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

void sample_plain(Arena &arena, const PlainInputs &in, PlainOutputs &out, hipStream_t s)
{
    const uint32_t T = in.count;
    const uint32_t chunk = std::min<uint32_t>(T, 1u << 21);
    uint64_t exp_size = std::max<uint64_t>(in.expected_size, 8);
    DevBuf<unsigned long long> hash;
    DevBuf<uint32_t> sizes, fill;
    DevBuf<unsigned long long> probed;
    DevBuf<uint2> entries;
    DevBuf<int4> itA, itB;
    DevBuf<uint32_t> np;
    DevBuf<int64_t> pbase, off;
    DevBuf<unsigned long long> ctr; // n_entries, n_items_out
    DevBuf<int> err;
    sizes.alloc(arena, chunk);
    fill.alloc(arena, chunk);
    probed.alloc(arena, chunk);
    off.alloc(arena, (size_t)chunk + 1);
    ctr.alloc(arena, 4);
    err.alloc(arena, 1);
    uint64_t hcap = 0, ecap = 0;
    auto size_buffers = [&](uint64_t exp_entries, uint64_t min_hcap) {
        uint64_t want_h = 1;
        while (want_h < std::max<uint64_t>(exp_entries * 5 / 2, min_hcap)) want_h <<= 1;
        const uint64_t want_e = exp_entries * 2 + (1u << 20);
        if (want_h > hcap) {
            hash.alloc(arena, want_h);
            hcap = want_h;
        }
        if (want_e > ecap) {
            entries.alloc(arena, want_e);
            itA.alloc(arena, want_e);
            itB.alloc(arena, want_e);
            np.alloc(arena, want_e);
            pbase.alloc(arena, want_e + 1);
            ecap = want_e;
        }
    };
    size_buffers((uint64_t)chunk * exp_size, 0);

    int64_t base = 0;
    out.levels = 0;
    for (uint32_t i0 = 0; i0 < T; i0 += chunk) {
        const uint32_t cn = std::min<uint32_t>(chunk, T - i0);
        unsigned long long ne = 0;
        for (int attempt = 0;; ++attempt) {
            hipLaunchKernelGGL(k_plain_fill<int>, dim3(1), dim3(64), 0, s, (uint64_t)1, err.ptr, 0);
            hipLaunchKernelGGL(k_plain_fill<unsigned long long>, dim3(gridp(hcap)), dim3(PLAIN_BLOCK), 0, s, hcap,
                               hash.ptr, HASH_EMPTY);
            hipLaunchKernelGGL(k_plain_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)4, ctr.ptr, 0ull);
            PlainCtx c;
            c.row_ptr = in.row_ptr;
            c.pairs = in.pairs;
            c.nquads = in.nquads;
            c.wbits = in.wbits;
            c.hash = hash.ptr;
            c.hmask = hcap - 1;
            c.sizes = sizes.ptr;
            c.probed = probed.ptr;
            c.entries = entries.ptr;
            c.n_entries = ctr.ptr + 0;
            c.entries_cap = ecap;
            c.items_out = itA.ptr;
            c.n_items_out = ctr.ptr + 1;
            c.items_cap = ecap;
            c.err = err.ptr;
            hipLaunchKernelGGL(k_plain_init, dim3(gridp(cn)), dim3(PLAIN_BLOCK), 0, s, cn, i0, in.rec, in.u1, c);
            SKIS_HIP_TRY(hipGetLastError());
            int4 *cur = itA.ptr, *nxt = itB.ptr;
            bool overflow = false;
            for (;;) {
                unsigned long long hv[2];
                int herr = 0;
                SKIS_HIP_TRY(hipMemcpyAsync(hv, ctr.ptr, sizeof(hv), hipMemcpyDeviceToHost, s));
                SKIS_HIP_TRY(hipMemcpyAsync(&herr, err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
                SKIS_HIP_TRY(hipStreamSynchronize(s));
                if (herr & 8) throw Error{SKIS_EHIP, "plain sampler: bounds check failed"};
                if (herr || hv[1] > ecap) {
                    overflow = true;
                    break;
                }
                const uint64_t n_items = hv[1];
                if (n_items == 0) break;
                ++out.levels;
                hipLaunchKernelGGL(k_plain_quads, dim3(gridp(n_items)), dim3(PLAIN_BLOCK), 0, s, (uint64_t)n_items, cur,
                                   np.ptr);
                excl_scan_u32_to_i64(arena, np.ptr, pbase.ptr, (int64_t)n_items, pbase.ptr + n_items, s);
                int64_t total = 0;
                SKIS_HIP_TRY(hipMemcpyAsync(&total, pbase.ptr + n_items, sizeof(total), hipMemcpyDeviceToHost, s));
                hipLaunchKernelGGL(k_plain_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)1, ctr.ptr + 1,
                                   0ull);
                SKIS_HIP_TRY(hipStreamSynchronize(s));
                c.items_out = nxt;
                const uint64_t wins = ((uint64_t)total + PLAIN_WINDOW - 1) / PLAIN_WINDOW;
                const unsigned ge =
                    (unsigned)std::min<uint64_t>(std::max<uint64_t>(wins, 1), (uint64_t)device_cu_count() * 16);
                hipLaunchKernelGGL(k_plain_expand, dim3(ge), dim3(PLAIN_BLOCK), 0, s, (uint64_t)n_items, cur,
                                   pbase.ptr, total, in.seed_lo, in.seed_hi, in.first_id + (uint64_t)i0, c);
                SKIS_HIP_TRY(hipGetLastError());
                std::swap(cur, nxt);
            }
            SKIS_HIP_TRY(hipMemcpyAsync(&ne, ctr.ptr, sizeof(ne), hipMemcpyDeviceToHost, s));
            SKIS_HIP_TRY(hipStreamSynchronize(s));
            if (!overflow) break;
            if (attempt == 6) throw Error{SKIS_ENOMEM, "plain sampler: chunk buffers kept overflowing"};
            // the chunk is a pure function of its sample ids: grow and run it again
            exp_size *= 4;
            size_buffers(std::max<uint64_t>((uint64_t)cn * exp_size, ne * 2), hcap * 2);
        }
        // chunk compaction (staging grows, keeping what earlier chunks wrote)
        if ((uint64_t)base + ne > in.staging->count) {
            DevBuf<int32_t> bigger;
            bigger.alloc(arena, std::max<uint64_t>(in.staging->count * 2, (uint64_t)base + ne + (1u << 20)));
            if (base > 0)
                SKIS_HIP_TRY(hipMemcpyAsync(bigger.ptr, in.staging->ptr, sizeof(int32_t) * (size_t)base,
                                            hipMemcpyDeviceToDevice, s));
            SKIS_HIP_TRY(hipStreamSynchronize(s));
            in.staging->swap(bigger);
        }
        excl_scan_u32_to_i64(arena, sizes.ptr, off.ptr, cn, off.ptr + cn, s);
        hipLaunchKernelGGL(k_plain_fill<uint32_t>, dim3(gridp(cn)), dim3(PLAIN_BLOCK), 0, s, (uint64_t)cn, fill.ptr, 0u);
        hipLaunchKernelGGL(k_plain_scatter, dim3(gridp(ne)), dim3(PLAIN_BLOCK), 0, s, (uint64_t)ne, entries.ptr, off.ptr,
                           base, fill.ptr, in.staging->ptr, (uint64_t)in.staging->count, err.ptr);
        hipLaunchKernelGGL(k_plain_meta, dim3(gridp(cn)), dim3(PLAIN_BLOCK), 0, s, cn, i0, sizes.ptr, probed.ptr, off.ptr,
                           base, in.out_size, in.out_off, in.out_probed, in.medium, in.n_medium, in.small_sort);
        SKIS_HIP_TRY(hipGetLastError());
        int herr = 0;
        SKIS_HIP_TRY(hipMemcpyAsync(&herr, err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        if (herr) throw Error{SKIS_ENOMEM, "plain sampler: staging too small"};
        base += (int64_t)ne;
    }
    out.entries = (uint64_t)base;
}

} // namespace skis
