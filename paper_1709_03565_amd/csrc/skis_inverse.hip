// skis_inverse.hip -- the node -> samples transpose of the sketch, H(v) = { j : v in R_j },
// used by the estimator (Eq. eq21) and the greedy (Eq. margin).  The transpose itself is a
// radix sort (skis_transpose.hip); this file adds the pick of the most frequent nodes, whose
// Delta the greedy keeps in LDS.
#include <algorithm>
#include <vector>

#include "skis_internal.h"

namespace skis {

constexpr int INV_HOT = 2048;            // hot nodes: the most frequent ones, at most this many

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
    if (T == 0 || sk.entries == 0) {
        hipLaunchKernelGGL(k_inv_fill<uint32_t>, dim3(grid_inv(n, 256)), dim3(256), 0, s, (uint64_t)n, cnt.ptr, 0u);
        SKIS_HIP_TRY(hipGetLastError());
        excl_scan_u32_to_i64(arena, cnt.ptr, sk.node_ptr.ptr, n, sk.node_ptr.ptr + n, s);
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        sk.has_inverse = true;
        return;
    }
    radix_transpose(arena, sk.sample_ptr.ptr, sk.nodes.ptr, sk.owner.count == sk.entries ? sk.owner.ptr : nullptr, T,
                    sk.entries, n, sk.node_ptr.ptr, sk.node_samples.ptr, cnt.ptr, s);
    sk.owner.reset();

    // hot nodes from the exact degrees: the smallest power-of-two threshold (at least 16
    // samples) that keeps at most INV_HOT nodes
    // cnt holds the exact degrees (the transpose counted them)
    DevBuf<unsigned long long> hist;
    hist.alloc(arena, 33);
    hipLaunchKernelGGL(k_inv_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)33, hist.ptr, 0ull);
    hipLaunchKernelGGL(k_inv_hist, dim3(grid_inv(n, 256)), dim3(256), 0, s, n, cnt.ptr, hist.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    unsigned long long hh[33];
    SKIS_HIP_TRY(hipMemcpyAsync(hh, hist.ptr, sizeof(hh), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    int bsel = 33;
    unsigned long long above = 0;
    for (int b = 32; b >= 4; --b) {
        if (above + hh[b] > (unsigned long long)INV_HOT) break;
        above += hh[b];
        bsel = b;
    }
    const uint32_t thr = bsel >= 32 ? 0xFFFFFFFFu : (1u << bsel);
    DevBuf<uint32_t> flag, rank, ntot;
    DevBuf<int32_t> &hot_id = sk.hot_id, &hot_node = sk.hot_node;
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
    sk.has_inverse = true;
}

} // namespace skis
