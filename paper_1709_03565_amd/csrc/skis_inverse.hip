// skis_inverse.hip -- the node -> samples transpose of the sketch, H(v) = { j : v in R_j },
// used by the estimator (Eq. eq21) and the greedy (Eq. margin).
//
// A few nodes sit in a large share of all samples (hubs of the reverse cascades), so a
// plain atomic histogram and scatter serialise on their counters.  Here the samples are cut
// into chunks; up to HOT frequent nodes, picked from a prefix of the sketch, are counted
// and placed per chunk in LDS, and every chunk gets its own write base for each of them
// from a column prefix sum over a chunk x HOT matrix.  Other nodes use global atomics.
// Lists come out in no particular order.
#include <algorithm>
#include <vector>

#include "skis_internal.h"

namespace skis {

constexpr int INV_HOT = 2048;            // hot nodes kept in LDS
constexpr uint32_t INV_CHUNK = 8192;     // samples per chunk
constexpr uint32_t INV_PREFIX = 65536;   // samples used to pick the hot nodes

__global__ __launch_bounds__(256) void k_inv_count_plain(uint64_t entries, const int32_t *__restrict__ nodes,
                                                         uint32_t *__restrict__ cnt)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < entries; p += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[nodes[p]], 1u);
}

// hist[b] = #{ v : floor(log2(cnt[v])) == b } for cnt[v] > 0
__global__ __launch_bounds__(256) void k_inv_hist(int32_t n, const uint32_t *__restrict__ cnt,
                                                  unsigned long long *__restrict__ hist)
{
    __shared__ unsigned int h[33];
    if (threadIdx.x < 33) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cnt[v];
        if (c) atomicAdd(&h[31 - __clz((int)c)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 33 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_inv_flags(int32_t n, const uint32_t *__restrict__ cnt, uint32_t thr,
                                                   uint32_t *__restrict__ flag)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = cnt[v] >= thr ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_inv_hot_ids(int32_t n, const uint32_t *__restrict__ flag,
                                                     const uint32_t *__restrict__ rank, int32_t *__restrict__ hot_id,
                                                     int32_t *__restrict__ hot_node)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (flag[v] && rank[v] < (uint32_t)INV_HOT) { // the threshold keeps at most INV_HOT
            hot_id[v] = (int32_t)rank[v];
            hot_node[rank[v]] = (int32_t)v;
        } else {
            hot_id[v] = -1;
        }
    }
}

// Counting pass: hot nodes per chunk in LDS (written to M[chunk][h]), the rest globally.
__global__ __launch_bounds__(256) void k_inv_count(uint64_t T, uint32_t nchunks, int nhot,
                                                   const int64_t *__restrict__ sptr, const int32_t *__restrict__ nodes,
                                                   const int32_t *__restrict__ hot_id, uint32_t *__restrict__ cnt,
                                                   uint32_t *__restrict__ M, unsigned long long *__restrict__ hot_total)
{
    __shared__ uint32_t hc[INV_HOT];
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        for (int h = threadIdx.x; h < nhot; h += 256) hc[h] = 0u;
        __syncthreads();
        const uint64_t j0 = (uint64_t)c * INV_CHUNK;
        const uint64_t j1 = std::min<uint64_t>(j0 + INV_CHUNK, T);
        const int64_t a = sptr[j0], b = sptr[j1];
        for (int64_t p = a + threadIdx.x; p < b; p += 256) {
            const int32_t v = nodes[p];
            const int32_t h = hot_id[v];
            if (h >= 0) atomicAdd(&hc[h], 1u);
            else atomicAdd(&cnt[v], 1u);
        }
        __syncthreads();
        for (int h = threadIdx.x; h < nhot; h += 256) {
            const uint32_t x = hc[h];
            M[(uint64_t)c * nhot + h] = x;
            if (x) atomicAdd(&hot_total[h], (unsigned long long)x);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_inv_hot_counts(int nhot, const int32_t *__restrict__ hot_node,
                                                        const unsigned long long *__restrict__ hot_total,
                                                        uint32_t *__restrict__ cnt)
{
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < nhot; h += gridDim.x * blockDim.x)
        cnt[hot_node[h]] = (uint32_t)hot_total[h];
}

// Per hot node, turn the column M[.][h] into write bases node_ptr[v_h] + prefix over chunks.
__global__ __launch_bounds__(256) void k_inv_hot_bases(uint32_t nchunks, int nhot, const int32_t *__restrict__ hot_node,
                                                       const int64_t *__restrict__ node_ptr, uint32_t *__restrict__ M,
                                                       int64_t *__restrict__ B)
{
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < nhot; h += gridDim.x * blockDim.x) {
        int64_t acc = node_ptr[hot_node[h]];
        for (uint32_t c = 0; c < nchunks; ++c) {
            const uint64_t i = (uint64_t)c * nhot + h;
            const uint32_t x = M[i];
            B[i] = acc;
            acc += x;
        }
    }
}

// Placement pass: same chunks; hot nodes take positions from LDS counters seeded with the
// chunk's bases, the rest from global per-node fill counters.
__global__ __launch_bounds__(256) void k_inv_scatter(uint64_t T, uint32_t nchunks, int nhot,
                                                     const int64_t *__restrict__ sptr, const int32_t *__restrict__ nodes,
                                                     const int32_t *__restrict__ hot_id,
                                                     const int64_t *__restrict__ node_ptr,
                                                     const int64_t *__restrict__ B, uint32_t *__restrict__ fill,
                                                     int32_t *__restrict__ ns)
{
    __shared__ unsigned long long hp[INV_HOT];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        for (int h = threadIdx.x; h < nhot; h += 256) hp[h] = (unsigned long long)B[(uint64_t)c * nhot + h];
        __syncthreads();
        const uint64_t j0 = (uint64_t)c * INV_CHUNK;
        const uint64_t j1 = std::min<uint64_t>(j0 + INV_CHUNK, T);
        for (uint64_t j = j0 + wid; j < j1; j += 4) {
            const int64_t a = sptr[j], b = sptr[j + 1];
            for (int64_t p = a + lane; p < b; p += 64) {
                const int32_t v = nodes[p];
                const int32_t h = hot_id[v];
                int64_t pos;
                if (h >= 0) pos = (int64_t)atomicAdd(&hp[h], 1ull);
                else pos = node_ptr[v] + (int64_t)atomicAdd(&fill[v], 1u);
                ns[pos] = (int32_t)j;
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_inv_fill(uint64_t count, T *__restrict__ p, T v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_inv(uint64_t items, int block, int per_cu = 16)
{
    uint64_t g = (items + block - 1) / block;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

void build_inverse(Sketch &sk, hipStream_t s)
{
    Arena &arena = sk.arena;
    const int32_t n = sk.n;
    const uint64_t T = sk.T;
    sk.node_ptr.alloc(arena, (size_t)n + 1);
    sk.node_samples.alloc(arena, (size_t)sk.entries);
    DevBuf<uint32_t> cnt;
    cnt.alloc(arena, (size_t)n);
    hipLaunchKernelGGL(k_inv_fill<uint32_t>, dim3(grid_inv(n, 256)), dim3(256), 0, s, (uint64_t)n, cnt.ptr, 0u);
    SKIS_HIP_TRY(hipGetLastError());
    if (T == 0 || sk.entries == 0) {
        excl_scan_u32_to_i64(arena, cnt.ptr, sk.node_ptr.ptr, n, sk.node_ptr.ptr + n, s);
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        sk.has_inverse = true;
        return;
    }

    // 1. hot nodes: the most frequent ones in a prefix of the sketch, at most INV_HOT
    const uint64_t pre = std::min<uint64_t>(T, INV_PREFIX);
    int64_t pre_entries = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&pre_entries, sk.sample_ptr.ptr + pre, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    hipLaunchKernelGGL(k_inv_count_plain, dim3(grid_inv(pre_entries, 256)), dim3(256), 0, s, (uint64_t)pre_entries,
                       sk.nodes.ptr, cnt.ptr);
    DevBuf<unsigned long long> hist;
    hist.alloc(arena, 33);
    hipLaunchKernelGGL(k_inv_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)33, hist.ptr, 0ull);
    hipLaunchKernelGGL(k_inv_hist, dim3(grid_inv(n, 256)), dim3(256), 0, s, n, cnt.ptr, hist.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    unsigned long long hh[33];
    SKIS_HIP_TRY(hipMemcpyAsync(hh, hist.ptr, sizeof(hh), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    // smallest power-of-two threshold (>= 16 occurrences in the prefix) that keeps <= INV_HOT nodes
    int bsel = 33;
    unsigned long long above = 0;
    for (int b = 32; b >= 4; --b) {
        if (above + hh[b] > (unsigned long long)INV_HOT) break;
        above += hh[b];
        bsel = b;
    }
    const uint32_t thr = bsel >= 32 ? 0xFFFFFFFFu : (1u << bsel);
    DevBuf<uint32_t> flag, rank, ntot;
    DevBuf<int32_t> &hot_id = sk.hot_id, &hot_node = sk.hot_node; // kept: the greedy uses them too
    flag.alloc(arena, n);
    rank.alloc(arena, n);
    ntot.alloc(arena, 1);
    hot_id.alloc(arena, n);
    hot_node.alloc(arena, INV_HOT);
    hipLaunchKernelGGL(k_inv_flags, dim3(grid_inv(n, 256)), dim3(256), 0, s, n, cnt.ptr, thr, flag.ptr);
    excl_scan<uint32_t>(arena, flag.ptr, rank.ptr, n, ntot.ptr, s);
    hipLaunchKernelGGL(k_inv_hot_ids, dim3(grid_inv(n, 256)), dim3(256), 0, s, n, flag.ptr, rank.ptr, hot_id.ptr,
                       hot_node.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    uint32_t nhot_u = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&nhot_u, ntot.ptr, sizeof(nhot_u), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    const int nhot = (int)std::min<uint32_t>(nhot_u, INV_HOT);
    if ((uint32_t)nhot != nhot_u) throw Error{SKIS_EHIP, "internal error: too many hot nodes"};
    sk.nhot = nhot;

    // 2. counts
    const uint32_t nchunks = (uint32_t)((T + INV_CHUNK - 1) / INV_CHUNK);
    const uint64_t mcount = (uint64_t)nchunks * (uint64_t)(nhot > 0 ? nhot : 1);
    DevBuf<uint32_t> M;
    DevBuf<int64_t> Bs;
    DevBuf<unsigned long long> hot_total;
    M.alloc(arena, mcount);
    Bs.alloc(arena, mcount);
    hot_total.alloc(arena, INV_HOT);
    hipLaunchKernelGGL(k_inv_fill<uint32_t>, dim3(grid_inv(n, 256)), dim3(256), 0, s, (uint64_t)n, cnt.ptr, 0u);
    hipLaunchKernelGGL(k_inv_fill<unsigned long long>, dim3(grid_inv(INV_HOT, 256)), dim3(256), 0, s,
                       (uint64_t)INV_HOT, hot_total.ptr, 0ull);
    const unsigned gc = std::min<unsigned>(nchunks, (unsigned)device_cu_count() * 8);
    hipLaunchKernelGGL(k_inv_count, dim3(gc), dim3(256), 0, s, T, nchunks, nhot, sk.sample_ptr.ptr, sk.nodes.ptr,
                       hot_id.ptr, cnt.ptr, M.ptr, hot_total.ptr);
    if (nhot > 0)
        hipLaunchKernelGGL(k_inv_hot_counts, dim3(grid_inv(nhot, 256)), dim3(256), 0, s, nhot, hot_node.ptr,
                           hot_total.ptr, cnt.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    // 3. offsets
    excl_scan_u32_to_i64(arena, cnt.ptr, sk.node_ptr.ptr, n, sk.node_ptr.ptr + n, s);
    if (nhot > 0)
        hipLaunchKernelGGL(k_inv_hot_bases, dim3(grid_inv(nhot, 64)), dim3(64), 0, s, nchunks, nhot, hot_node.ptr,
                           sk.node_ptr.ptr, M.ptr, Bs.ptr);
    // 4. placement
    hipLaunchKernelGGL(k_inv_fill<uint32_t>, dim3(grid_inv(n, 256)), dim3(256), 0, s, (uint64_t)n, cnt.ptr, 0u);
    hipLaunchKernelGGL(k_inv_scatter, dim3(gc), dim3(256), 0, s, T, nchunks, nhot, sk.sample_ptr.ptr, sk.nodes.ptr,
                       hot_id.ptr, sk.node_ptr.ptr, Bs.ptr, cnt.ptr, sk.node_samples.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    sk.has_inverse = true;
}

} // namespace skis
