// skis_query.hip -- queries on the device-resident sketch:
//   k_estimate   Eq. (eq21): Cov(S) by marking the samples of every v in S in a bitmap over
//                the T samples (a sample counts once, when its bit first flips), and
//                I_hat(S) = fl(fl(Cov * Gamma) / T) + sum_{v in S} q_v (compensated sum).
//   k_greedy_*   Alg. 3: the node of largest gain fl(fl(Delta * Gamma) / T) + q (Eq. margin),
//                smallest id on ties; Delta kept exact by decrementing the members of every
//                newly covered sample.
#include "skis_internal.h"
#include "skis_query.h"

#include <algorithm>
#include <vector>

namespace skis {

__device__ __forceinline__ void neumaier_add(double &s, double &c, double x)
{
    const double t = __dadd_rn(s, x);
    if (fabs(s) >= fabs(x)) c = __dadd_rn(c, __dadd_rn(__dsub_rn(s, t), x));
    else c = __dadd_rn(c, __dadd_rn(__dsub_rn(x, t), s));
    s = t;
}

template <int NT>
__device__ void bitonic_sort_lds(int32_t *buf, int P)
{
    for (int k = 2; k <= P; k <<= 1) {
        for (int d = k >> 1; d > 0; d >>= 1) {
            for (int i = threadIdx.x; i < P; i += NT) {
                const int ixj = i ^ d;
                if (ixj > i) {
                    const int32_t x = buf[i], y = buf[ixj];
                    const bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        buf[i] = y;
                        buf[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Flips the bit of sample j in bm for every lane of the wave with in = true and returns the
// bits this lane flipped; every lane of the wave must call it.  A sample list is sorted by
// sample id and a wave walks consecutive entries, so on a dense list (a hub's) neighbouring
// lanes often share a bitmap word.  When any do, the bits of lanes with the same word are
// OR-ed within aligned groups of 8 lanes by a segmented scan (a lane takes the running OR of
// lane - d in its group when their words agree; a run of equal words is contiguous, and lanes
// of another run with the same word only add bits of that word), and the last lane of each
// run in a group sets them with one atomicOr.  Atomics on one word are serialised, so every
// flip is counted once.  When no neighbours share a word, each lane flips its own bit.
__device__ __forceinline__ unsigned long long flip_bits_wave(uint32_t *bm, int32_t j, bool in)
{
    const int lane = threadIdx.x & 63;
    const uint32_t w = (uint32_t)j >> 5;
    uint32_t acc = in ? 1u << (j & 31) : 0u;
    // the shuffle runs on every lane: under a mask it would read 0 from the masked lane 63
    const uint32_t nw = __shfl_down(w, 1, 64);
    const bool same_next = lane < 63 && nw == w;
    bool last = true;
    if (__ballot(same_next) != 0ull) { // wave-uniform
#pragma unroll
        for (int d = 1; d < 8; d <<= 1) {
            const uint32_t ow = __shfl_up(w, d, 64), oa = __shfl_up(acc, d, 64);
            if ((lane & 7) >= d && ow == w) acc |= oa;
        }
        last = (lane & 7) == 7 || !same_next;
    }
    if (!last || !acc) return 0ull;
    const uint32_t old = atomicOr(&bm[w], acc);
    return (unsigned long long)__popc(acc & ~old);
}

// One workgroup per query.  The set is taken in chunks of EST_MAX_SET entries; each chunk is
// sorted and deduplicated in LDS.  LARGE workgroups (sets above one chunk) also keep a
// bitmap of n bits that drops ids already met in an earlier chunk.  The distinct members'
// q values are summed (compensated, in a fixed order) and their sample lists H(v) are
// walked flat across the workgroup, flipping one bit per sample in a bitmap of T bits;
// Cov(S) is the number of flips.
template <bool LARGE>
__global__ __launch_bounds__(EST_BLOCK) void k_estimate(const int64_t *__restrict__ qlist, int64_t q0,
                                                        const int64_t *__restrict__ set_ptr,
                                                        const int32_t *__restrict__ set_nodes, int32_t n, uint64_t T,
                                                        double Gamma, const double *__restrict__ qv,
                                                        const int64_t *__restrict__ node_ptr,
                                                        const int32_t *__restrict__ node_samples,
                                                        uint32_t *__restrict__ bitmaps, uint64_t wordsT,
                                                        uint32_t *__restrict__ nodebits, uint64_t wordsN,
                                                        unsigned long long *__restrict__ cov_out,
                                                        double *__restrict__ est_out, int *__restrict__ err)
{
    __shared__ int32_t buf[EST_MAX_SET];
    __shared__ int64_t dbase[EST_MAX_SET + 1];
    __shared__ int32_t s_scan[EST_BLOCK / 64 + 1];
    __shared__ int64_t s_scan64[EST_BLOCK / 64 + 1];
    __shared__ double ps[EST_BLOCK], pc[EST_BLOCK];
    __shared__ unsigned long long s_cov[EST_BLOCK / 64];
    __shared__ int s_bad;

    const int64_t qi = LARGE ? qlist[q0 + blockIdx.x] : q0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t a = set_ptr[qi], b = set_ptr[qi + 1];
    const int64_t k = b - a;
    if (k < 0) {
        if (tid == 0) atomicOr(err, 1);
        return;
    }
    if (!LARGE && k > EST_MAX_SET) return; // taken by the LARGE launch
    uint32_t *bm = bitmaps + (uint64_t)blockIdx.x * wordsT;
    uint32_t *nb = LARGE ? nodebits + (uint64_t)blockIdx.x * wordsN : nullptr;
    constexpr int IPT = EST_MAX_SET / EST_BLOCK;

    double sq = 0.0, cq = 0.0;
    unsigned long long local = 0;
    int nu = 0, maxnu = 0; // maxnu: threads at or past it never took a member (their sums are +0)
    int64_t E = 0;
    for (int64_t c0 = a; c0 < b; c0 += EST_MAX_SET) {
        const int kc = (int)((b - c0) < EST_MAX_SET ? (b - c0) : EST_MAX_SET);
        if (tid == 0) s_bad = 0;
        __syncthreads();
        int P = 1;
        while (P < kc) P <<= 1;
        for (int t = tid; t < P; t += EST_BLOCK) {
            int32_t v = INT32_MAX;
            if (t < kc) {
                v = set_nodes[c0 + t];
                if (v < 0 || v >= n) {
                    s_bad = 1;
                    v = INT32_MAX;
                }
            }
            buf[t] = v;
        }
        __syncthreads();
        if (s_bad) {
            if (tid == 0) atomicOr(err, 4);
            return;
        }
        if (P > 1) bitonic_sort_lds<EST_BLOCK>(buf, P);

        // distinct members of the chunk (and, for LARGE, not met before), compacted in order
        int32_t mine[IPT];
        int flags = 0, cntu = 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int t = tid * IPT + r;
            const int32_t v = t < kc ? buf[t] : INT32_MAX;
            mine[r] = v;
            bool u = t < kc && (t == 0 || buf[t - 1] != v);
            if (LARGE && u) {
                const uint32_t bit = 1u << (v & 31);
                u = !(atomicOr(&nb[v >> 5], bit) & bit);
            }
            flags |= (u ? 1 : 0) << r;
            cntu += u ? 1 : 0;
        }
        int pos = block_excl_scan<EST_BLOCK, int>(cntu, s_scan, &nu);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (flags >> r & 1) buf[pos++] = mine[r];
        __syncthreads();

        if (qv)
            for (int t = tid; t < nu; t += EST_BLOCK) neumaier_add(sq, cq, qv[buf[t]]);
        maxnu = nu > maxnu ? nu : maxnu;
        int64_t dl[IPT];
        int64_t acc = 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int t = tid * IPT + r;
            int64_t d = 0;
            if (t < nu) {
                const int32_t v = buf[t];
                d = node_ptr[v + 1] - node_ptr[v];
            }
            dl[r] = acc;
            acc += d;
        }
        const int64_t ex = block_excl_scan<EST_BLOCK, int64_t>(acc, s_scan64, &E);
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int t = tid * IPT + r;
            if (t < nu) dbase[t] = ex + dl[r];
        }
        if (tid == 0) dbase[nu] = E;
        __syncthreads();
        // EST_WALK entries per thread and round, their loads issued together; a wave takes 64
        // consecutive entries and flips their bits with one atomic per bitmap word it meets.
        // The rounds are the same for the whole wave (the flips shuffle across it); a lane past
        // E repeats entry E - 1 (in bounds) and flips no bit.
        for (int64_t i0 = tid; i0 - (tid & 63) < E; i0 += (int64_t)EST_BLOCK * EST_WALK) { // wave-uniform
            int64_t ix[EST_WALK];
            int lv[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) {
                const int64_t idx = i0 + (int64_t)u * EST_BLOCK;
                ix[u] = idx < E ? idx : E - 1;
                int lo = 0, hi = nu - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (dbase[mid] <= ix[u]) lo = mid; else hi = mid - 1;
                }
                lv[u] = lo;
            }
            int64_t np[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) np[u] = node_ptr[buf[lv[u]]];
            int32_t jv[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) jv[u] = node_samples[np[u] + (ix[u] - dbase[lv[u]])];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) local += flip_bits_wave(bm, jv[u], i0 + (int64_t)u * EST_BLOCK < E);
        }
        __syncthreads();
    }

    ps[tid] = sq;
    pc[tid] = cq;
    local = wave_sum(local);
    if ((tid & 63) == 0) s_cov[tid >> 6] = local;
    __syncthreads();
    if (tid == 0) {
        unsigned long long c = 0;
        for (int w = 0; w < EST_BLOCK / 64; ++w) c += s_cov[w];
        double s = 0.0, cc = 0.0;
        // adding the +0 partials of the threads past maxnu would change neither s nor cc
        const int tq = maxnu < EST_BLOCK ? maxnu : EST_BLOCK;
        for (int t = 0; t < tq; ++t) {
            neumaier_add(s, cc, ps[t]);
            neumaier_add(s, cc, pc[t]);
        }
        const double first = T > 0 ? __ddiv_rn(__dmul_rn((double)c, Gamma), (double)T) : 0.0;
        cov_out[qi] = c;
        est_out[qi] = __dadd_rn(first, __dadd_rn(s, cc));
    }
    // leave the bitmaps clear for the next query
    if (LARGE) {
        for (uint64_t w = tid; w < wordsT; w += EST_BLOCK) bm[w] = 0u;
        for (int64_t t = a + tid; t < b; t += EST_BLOCK) nb[set_nodes[t] >> 5] = 0u;
    } else {
        // one chunk: buf and dbase still hold it; the same rounds as the walk (a lane past E
        // clears the word of entry E - 1 once more)
        for (int64_t i0 = tid; i0 - (tid & 63) < E; i0 += (int64_t)EST_BLOCK * EST_WALK) { // wave-uniform
            int64_t ix[EST_WALK];
            int lv[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) {
                const int64_t idx = i0 + (int64_t)u * EST_BLOCK;
                ix[u] = idx < E ? idx : E - 1;
                int lo = 0, hi = nu - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (dbase[mid] <= ix[u]) lo = mid; else hi = mid - 1;
                }
                lv[u] = lo;
            }
            int64_t np[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) np[u] = node_ptr[buf[lv[u]]];
            int32_t jv[EST_WALK];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) jv[u] = node_samples[np[u] + (ix[u] - dbase[lv[u]])];
#pragma unroll
            for (int u = 0; u < EST_WALK; ++u) { // the last lane of each run of equal words clears it
                const uint32_t w = (uint32_t)jv[u] >> 5, nw = __shfl_down(w, 1, 64);
                if ((threadIdx.x & 63) == 63 || nw != w) bm[w] = 0u;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Greedy (Alg. 3) with exact marginal coverage.  delta[v] = #{ j in H(v) : j not covered }.
// Each round: k_greedy_argmax picks the node of largest gain fl(fl(delta * Gamma) / T) + q_v
// (Eq. margin; smallest id on ties); k_greedy_cover sets the covered bits of H(v*) and lowers
// delta of every member of the samples it newly covers, or, when they are many,
// k_greedy_recount counts delta afresh from the lists.  Three launches per round and no host
// synchronisation inside the k rounds.
// ---------------------------------------------------------------------------------------
// A round that covers more than T / RECOUNT_DIV samples recounts Delta of every node from
// its list instead of decrementing the members of each newly covered sample.
constexpr uint64_t RECOUNT_DIV = 32;
constexpr int RECOUNT_SPAN = 1024; // list entries per recount work item
constexpr int RECOUNT_LANES = 16;  // lanes per work item
constexpr int RECOUNT_UNROLL = 8;  // loads in flight per lane

__device__ __forceinline__ bool heavy_round(const GreedyState *st, uint64_t T)
{
    return st->vstar >= 0 && st->dstar > T / RECOUNT_DIV;
}

__device__ __forceinline__ double gain_of(int64_t d, uint64_t T, double Gamma, double q)
{
    return __dadd_rn(T > 0 ? __ddiv_rn(__dmul_rn((double)d, Gamma), (double)T) : 0.0, q);
}

__device__ __forceinline__ bool better(double g, int32_t v, double bg, int32_t bv)
{
    return bv < 0 || g > bg || (g == bg && v < bv);
}

__global__ __launch_bounds__(256) void k_greedy_init(int32_t n, const int64_t *__restrict__ node_ptr,
                                                     int32_t *__restrict__ delta, uint8_t *__restrict__ chosen)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        delta[v] = (int32_t)(node_ptr[v + 1] - node_ptr[v]);
        chosen[v] = 0;
    }
}

// (g, v) maximum under the order "larger gain, then smaller id" (a total order on the
// valid pairs, so any reduction tree gives the same winner); v < 0 marks an empty slot.
__device__ __forceinline__ void wave_best(double &g, int32_t &v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const double og = __shfl_xor(g, d, 64);
        const int32_t ov = __shfl_xor(v, d, 64);
        if (ov >= 0 && better(og, ov, g, v)) {
            g = og;
            v = ov;
        }
    }
}

// Workgroup-wide winner of 256 threads; every thread gets it.
__device__ __forceinline__ void block_best(double &g, int32_t &v, double *sg, int32_t *sv)
{
    wave_best(g, v);
    if ((threadIdx.x & 63) == 0) {
        sg[threadIdx.x >> 6] = g;
        sv[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    g = sg[0];
    v = sv[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
        if (sv[w] >= 0 && better(sg[w], sv[w], g, v)) {
            g = sg[w];
            v = sv[w];
        }
    __syncthreads();
}

// Each thread scans ARGMAX_PER nodes of its workgroup's tile, all loads issued before the
// gains are formed; the last workgroup to finish reduces the per-workgroup winners.
constexpr int ARGMAX_PER = 16;

// delta lives in two buffers: a round that recounts writes the spare one (kept zero), and
// the next argmax switches to it and zeroes the one it leaves as it scans.
__global__ __launch_bounds__(256) void k_greedy_argmax(int32_t n, int round, uint64_t T, double Gamma,
                                                       int32_t *__restrict__ delta0, int32_t *__restrict__ delta1,
                                                       const double *__restrict__ qv,
                                                       uint8_t *__restrict__ chosen, double *__restrict__ part_g,
                                                       int32_t *__restrict__ part_v, GreedyState *__restrict__ st,
                                                       int32_t *__restrict__ seeds,
                                                       unsigned long long *__restrict__ marg)
{
    __shared__ double sg[4];
    __shared__ int32_t sv[4];
    __shared__ bool last;
    const bool recounted = heavy_round(st, T); // the previous round (st is rewritten by the last block)
    const int cur = st->cur ^ (recounted ? 1 : 0);
    const int32_t *delta = cur ? delta1 : delta0;
    int32_t *spare = cur ? delta0 : delta1;
    double bg = 0.0;
    int32_t bv = -1;
    for (int64_t v0 = (int64_t)blockIdx.x * 256 * ARGMAX_PER + threadIdx.x; v0 < n;
         v0 += (int64_t)gridDim.x * 256 * ARGMAX_PER) {
        int32_t d[ARGMAX_PER];
        double q[ARGMAX_PER];
        uint8_t c[ARGMAX_PER];
#pragma unroll
        for (int u = 0; u < ARGMAX_PER; ++u) {
            const int64_t v = v0 + (int64_t)u * 256;
            const bool in = v < n;
            c[u] = in ? chosen[v] : (uint8_t)1;
            d[u] = in ? delta[v] : 0;
            q[u] = in && qv ? qv[v] : 0.0;
            if (recounted && in) spare[v] = 0;
        }
#pragma unroll
        for (int u = 0; u < ARGMAX_PER; ++u) {
            if (c[u]) continue;
            const int32_t v = (int32_t)(v0 + (int64_t)u * 256);
            const double g = gain_of(d[u], T, Gamma, q[u]);
            if (better(g, v, bg, bv)) {
                bg = g;
                bv = v;
            }
        }
    }
    block_best(bg, bv, sg, sv);
    if (threadIdx.x == 0) {
        part_g[blockIdx.x] = bg;
        part_v[blockIdx.x] = bv;
        __threadfence();
        last = atomicAdd(&st->done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    bg = 0.0;
    bv = -1;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += 256) {
        const int32_t pv = __hip_atomic_load(&part_v[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double pg = __longlong_as_double((long long)__hip_atomic_load(
            reinterpret_cast<unsigned long long *>(&part_g[b]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (pv >= 0 && better(pg, pv, bg, bv)) {
            bg = pg;
            bv = pv;
        }
    }
    block_best(bg, bv, sg, sv);
    if (threadIdx.x == 0) {
        st->done = 0u;
        if (recounted) {
            st->shrunk = 1u; // the previous round rewrote the spans
            st->cur = cur;
        }
        if (bv < 0) { // nothing left to pick (cannot happen for k <= n)
            st->vstar = -1;
            return;
        }
        st->vstar = bv;
        const int32_t d = delta[bv];
        st->dstar = (unsigned long long)d;
        seeds[round] = bv;
        marg[round] = (unsigned long long)d;
        chosen[bv] = 1;
        st->cov += (unsigned long long)d;
    }
}

// Covers H(v*).  H(v*) is in ascending sample order, so each lane takes a run of MARK_RUN
// consecutive entries and sets the bits of one bitmap word with one atomicOr.  In a round that
// does not recount, each wave queues the samples it newly covered in LDS and lowers delta of
// every member of each (16 lanes per sample); the most frequent nodes (the transpose's hot
// list) are decremented in LDS per workgroup and flushed once, so hubs do not serialise on
// one counter.  Integer updates commute, so delta and the picks are exact.  The number of
// samples a round newly covers is delta of its pick, known before the round starts.
constexpr int MARK_RUN = 8;

__global__ __launch_bounds__(256) void k_greedy_cover(const GreedyState *__restrict__ st, uint64_t T,
                                                      const int64_t *__restrict__ node_ptr,
                                                      const int32_t *__restrict__ node_samples,
                                                      uint32_t *__restrict__ covered,
                                                      const int64_t *__restrict__ sptr,
                                                      const int32_t *__restrict__ nodes,
                                                      const int32_t *__restrict__ hot_id,
                                                      const int32_t *__restrict__ hot_node, int nhot,
                                                      int32_t *__restrict__ delta0, int32_t *__restrict__ delta1)
{
    __shared__ int32_t hd[GREEDY_HOT];
    __shared__ uint32_t queue[4][64 * MARK_RUN];
    const int32_t v = st->vstar;
    if (v < 0) return;
    const bool update = !heavy_round(st, T);
    int32_t *delta = st->cur ? delta1 : delta0;
    if (update)
        for (int h = threadIdx.x; h < nhot; h += 256) hd[h] = 0;
    __syncthreads();
    const int64_t a = node_ptr[v], b = node_ptr[v + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t *q = queue[wid];
    for (int64_t c0 = a + wave * 64 * MARK_RUN; c0 < b; c0 += nwaves * 64 * MARK_RUN) { // uniform per wave
        const int64_t r0 = c0 + (int64_t)lane * MARK_RUN;
        int32_t js[MARK_RUN];
        int n = 0;
#pragma unroll
        for (int k = 0; k < MARK_RUN; ++k) {
            js[k] = r0 + k < b ? node_samples[r0 + k] : -1;
            n += js[k] >= 0 ? 1 : 0;
        }
        uint32_t fresh = 0; // bit k: js[k] newly covered
        int k = 0;
        while (k < n) { // one word at a time
            const int32_t word = js[k] >> 5;
            uint32_t bits = 0;
            int k1 = k;
            while (k1 < n && (js[k1] >> 5) == word) bits |= 1u << (js[k1++] & 31);
            const uint32_t newb = bits & ~atomicOr(&covered[word], bits);
            for (int t = k; t < k1; ++t)
                if (newb & (1u << (js[t] & 31))) fresh |= 1u << t;
            k = k1;
        }
        if (!update) continue;
        const int cnt = __popc(fresh);
        const int incl = wave_incl_scan(cnt);
        const int tot = (int)lane_value((uint32_t)incl, 63);
        if (!tot) continue;
        int pos = incl - cnt;
#pragma unroll
        for (int t = 0; t < MARK_RUN; ++t)
            if (fresh & (1u << t)) q[pos++] = (uint32_t)js[t];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int g = lane >> 4, gl = lane & 15; // 4 samples at a time, 16 lanes each
        for (int i0 = 0; i0 < tot; i0 += 4) {
            const int i = i0 + g;
            if (i >= tot) continue;
            const uint32_t j = q[i];
            const int64_t sa = sptr[j], sb = sptr[j + 1];
            for (int64_t t = sa + gl; t < sb; t += 16) {
                const int32_t u = nodes[t];
                const int32_t h = hot_id ? hot_id[u] : -1;
                if (h >= 0) atomicSub(&hd[h], 1);
                else atomicSub(&delta[u], 1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); // the queue is reused next
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (!update) return;
    __syncthreads();
    for (int h = threadIdx.x; h < nhot; h += 256)
        if (hd[h]) atomicAdd(&delta[hot_node[h]], hd[h]);
}

// Work items for the recount: each node's list cut into spans of RECOUNT_SPAN entries.
__global__ __launch_bounds__(256) void k_recount_items_count(int32_t n, const int64_t *__restrict__ node_ptr,
                                                             uint32_t *__restrict__ nitems)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = node_ptr[v + 1] - node_ptr[v];
        nitems[v] = (uint32_t)((d + RECOUNT_SPAN - 1) / RECOUNT_SPAN);
    }
}

__global__ __launch_bounds__(256) void k_recount_items_fill(int32_t n, const int64_t *__restrict__ node_ptr,
                                                            const uint32_t *__restrict__ nitems,
                                                            const int64_t *__restrict__ ioff,
                                                            RecountItem *__restrict__ items)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = node_ptr[v], d = node_ptr[v + 1] - a;
        for (uint32_t c = 0; c < nitems[v]; ++c) {
            RecountItem w;
            w.p0 = a + (int64_t)c * RECOUNT_SPAN;
            w.len = (int32_t)min<int64_t>(RECOUNT_SPAN, d - (int64_t)c * RECOUNT_SPAN);
            w.v = (int32_t)v;
            items[ioff[v] + c] = w;
        }
    }
}

// delta[v] += #{ j in span : j not covered }, and the span is cut down to those samples:
// the first heavy round reads node v's list from the sketch and writes the uncovered part
// to the same offsets of `work`; later heavy rounds read and rewrite `work` in place (a kept
// entry only moves to a lower position, after every load of its batch).  The order within
// a span stays ascending.  RECOUNT_LANES lanes per span, RECOUNT_UNROLL list loads and then
// as many bitmap loads in flight per lane.
__global__ __launch_bounds__(256) void k_greedy_recount(const GreedyState *__restrict__ st, uint64_t T,
                                                        uint64_t nitems, RecountItem *__restrict__ items,
                                                        const int32_t *node_samples, int32_t *work,
                                                        const uint32_t *__restrict__ covered,
                                                        int32_t *__restrict__ delta0, int32_t *__restrict__ delta1)
{
    if (!heavy_round(st, T)) return;
    int32_t *delta = st->cur ? delta0 : delta1; // the spare buffer, all zero; the next argmax switches
    const int32_t *src = st->shrunk ? work : node_samples;
    constexpr int G = 64 / RECOUNT_LANES;
    const int lane = threadIdx.x & 63, grp = lane / RECOUNT_LANES, t = lane % RECOUNT_LANES;
    const uint64_t below = (1ull << t) - 1ull;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t b0 = wave * G; b0 < nitems; b0 += nwaves * G) { // uniform over the wave
        const uint64_t it = b0 + grp;
        RecountItem w;
        w.p0 = 0;
        w.len = 0;
        w.v = -1;
        if (it < nitems) w = items[it];
        int kept = 0; // same in every lane of the group
        for (int q0 = 0; q0 < w.len; q0 += RECOUNT_LANES * RECOUNT_UNROLL) {
            int32_t js[RECOUNT_UNROLL];
#pragma unroll
            for (int u = 0; u < RECOUNT_UNROLL; ++u) {
                const int q = q0 + u * RECOUNT_LANES + t;
                js[u] = q < w.len ? src[w.p0 + q] : -1;
            }
            uint32_t wd[RECOUNT_UNROLL];
#pragma unroll
            for (int u = 0; u < RECOUNT_UNROLL; ++u) wd[u] = js[u] >= 0 ? covered[js[u] >> 5] : 0xffffffffu;
#pragma unroll
            for (int u = 0; u < RECOUNT_UNROLL; ++u) {
                const bool keep = !((wd[u] >> (js[u] & 31)) & 1u);
                const uint64_t m = (__ballot(keep) >> (grp * RECOUNT_LANES)) & 0xffffull;
                if (keep) work[w.p0 + kept + __popcll(m & below)] = js[u];
                kept += __popcll(m);
            }
        }
        if (t == 0 && it < nitems) {
            items[it].len = kept;
            if (kept) atomicAdd(&delta[w.v], kept);
        }
    }
}

// second term of Eq. margin summed over the k picks (each node is picked at most once)
__global__ __launch_bounds__(256) void k_greedy_final(int32_t k, uint64_t T, double Gamma,
                                                      const int32_t *__restrict__ seeds, const double *__restrict__ qv,
                                                      GreedyState *__restrict__ st)
{
    __shared__ double ps[256], pc[256];
    double s = 0.0, c = 0.0;
    if (qv)
        for (int32_t r = threadIdx.x; r < k; r += 256) neumaier_add(s, c, qv[seeds[r]]);
    ps[threadIdx.x] = s;
    pc[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tc = 0.0;
        for (int t = 0; t < 256; ++t) {
            neumaier_add(ts, tc, ps[t]);
            neumaier_add(ts, tc, pc[t]);
        }
        const double first = T > 0 ? __ddiv_rn(__dmul_rn((double)st->cov, Gamma), (double)T) : 0.0;
        st->est = __dadd_rn(first, __dadd_rn(ts, tc));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_q(uint64_t count, T *__restrict__ p, T v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned gridq(uint64_t items, int block, int per_cu = 8)
{
    uint64_t g = (items + block - 1) / block;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

void estimate_batch(const Sketch &sk, QueryScratch &qs, int32_t Q, const int64_t *set_ptr, const int32_t *set_nodes,
                    uint64_t *cov, double *est, hipStream_t s)
{
    Arena &arena = const_cast<Arena &>(sk.arena);
    // set sizes on the host: argument checks and the list of sets above one LDS chunk
    std::vector<int64_t> hptr((size_t)Q + 1);
    SKIS_HIP_TRY(hipMemcpyAsync(hptr.data(), set_ptr, sizeof(int64_t) * ((size_t)Q + 1), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int64_t> large;
    for (int32_t i = 0; i < Q; ++i) {
        const int64_t k = hptr[i + 1] - hptr[i];
        if (k < 0 || hptr[i] < 0) throw Error{SKIS_EINVAL, "set_ptr must be nondecreasing from 0"};
        if (k > EST_MAX_SET) large.push_back(i);
    }
    if (hptr[Q] > 0 && !set_nodes) throw Error{SKIS_EINVAL, "set_nodes must not be NULL"};

    const uint64_t wordsT = (sk.T + 31) / 32;
    const uint64_t per = wordsT ? wordsT : 1;
    // bitmaps for up to `batch` queries at a time, about 256 MiB
    uint64_t batch = (256ull << 20) / (per * 4);
    if (batch < 1) batch = 1;
    if (batch > 4096) batch = 4096;
    if (batch > (uint64_t)Q) batch = (uint64_t)Q;
    if (qs.bitmap_words < batch * per) {
        qs.bitmaps.alloc(arena, batch * per);
        qs.bitmap_words = batch * per;
        hipLaunchKernelGGL(k_fill_q<uint32_t>, dim3(gridq(batch * per, 256)), dim3(256), 0, s, batch * per,
                           qs.bitmaps.ptr, 0u);
        SKIS_HIP_TRY(hipGetLastError());
    }
    if (!qs.err.ptr) qs.err.alloc(arena, 1);
    hipLaunchKernelGGL(k_fill_q<int>, dim3(1), dim3(64), 0, s, (uint64_t)1, qs.err.ptr, 0);
    for (int64_t q0 = 0; q0 < Q; q0 += (int64_t)batch) {
        const int64_t nq = (Q - q0) < (int64_t)batch ? (Q - q0) : (int64_t)batch;
        hipLaunchKernelGGL(k_estimate<false>, dim3((unsigned)nq), dim3(EST_BLOCK), 0, s, (const int64_t *)nullptr, q0,
                           set_ptr, set_nodes, sk.n, sk.T, sk.est_scale(), sk.est_q(), sk.node_ptr.ptr, sk.node_samples.ptr,
                           qs.bitmaps.ptr, per, (uint32_t *)nullptr, (uint64_t)0,
                           reinterpret_cast<unsigned long long *>(cov), est, qs.err.ptr);
        SKIS_HIP_TRY(hipGetLastError());
    }
    if (!large.empty()) {
        const uint64_t wordsN = ((uint64_t)sk.n + 31) / 32;
        const uint64_t group = std::min<uint64_t>(std::min<uint64_t>(batch, 64), large.size());
        DevBuf<int64_t> qlist;
        DevBuf<uint32_t> nodebits;
        qlist.alloc(arena, large.size());
        nodebits.alloc(arena, group * wordsN);
        SKIS_HIP_TRY(hipMemcpyAsync(qlist.ptr, large.data(), sizeof(int64_t) * large.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_fill_q<uint32_t>, dim3(gridq(group * wordsN, 256)), dim3(256), 0, s, group * wordsN,
                           nodebits.ptr, 0u);
        for (uint64_t g0 = 0; g0 < large.size(); g0 += group) {
            const uint64_t ng = std::min<uint64_t>(group, large.size() - g0);
            hipLaunchKernelGGL(k_estimate<true>, dim3((unsigned)ng), dim3(EST_BLOCK), 0, s,
                               (const int64_t *)qlist.ptr, (int64_t)g0, set_ptr, set_nodes, sk.n, sk.T, sk.est_scale(),
                               sk.est_q(), sk.node_ptr.ptr, sk.node_samples.ptr, qs.bitmaps.ptr, per, nodebits.ptr,
                               wordsN, reinterpret_cast<unsigned long long *>(cov), est, qs.err.ptr);
            SKIS_HIP_TRY(hipGetLastError());
        }
        SKIS_HIP_TRY(hipStreamSynchronize(s));
    }
    int herr = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&herr, qs.err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (herr) {
        // a workgroup that stopped early may have left bits set: clear all scratch
        hipLaunchKernelGGL(k_fill_q<uint32_t>, dim3(gridq(qs.bitmap_words, 256)), dim3(256), 0, s, qs.bitmap_words,
                           qs.bitmaps.ptr, 0u);
        SKIS_HIP_TRY(hipStreamSynchronize(s));
    }
    if (herr & 1) throw Error{SKIS_EINVAL, "set_ptr must be nondecreasing"};
    if (herr & 4) throw Error{SKIS_EINVAL, "a seed set holds a node id outside [0, n)"};
}

void estimate_launch(const Sketch &sk, int32_t nq, const int64_t *set_ptr, const int32_t *set_nodes,
                     const int64_t *large, int32_t nlarge, uint32_t *bitmaps, uint64_t bitmap_words,
                     uint32_t *nodebits, unsigned long long *cov, double *est, int *err, hipStream_t s)
{
    const uint64_t per = bitmap_words;
    if (nq > 0) {
        hipLaunchKernelGGL(k_estimate<false>, dim3((unsigned)nq), dim3(EST_BLOCK), 0, s, (const int64_t *)nullptr,
                           (int64_t)0, set_ptr, set_nodes, sk.n, sk.T, sk.est_scale(), sk.est_q(), sk.node_ptr.ptr,
                           sk.node_samples.ptr, bitmaps, per, (uint32_t *)nullptr, (uint64_t)0, cov, est, err);
        SKIS_HIP_TRY(hipGetLastError());
    }
    if (nlarge > 0) {
        const uint64_t wordsN = ((uint64_t)sk.n + 31) / 32;
        hipLaunchKernelGGL(k_estimate<true>, dim3((unsigned)nlarge), dim3(EST_BLOCK), 0, s, large, (int64_t)0,
                           set_ptr, set_nodes, sk.n, sk.T, sk.est_scale(), sk.est_q(), sk.node_ptr.ptr, sk.node_samples.ptr,
                           bitmaps, per, nodebits, wordsN, cov, est, err);
        SKIS_HIP_TRY(hipGetLastError());
    }
}

void estimate_launch_small(const Sketch &sk, int64_t q0, int32_t nq, const int64_t *set_ptr,
                           const int32_t *set_nodes, uint32_t *bitmaps, uint64_t bitmap_words,
                           unsigned long long *cov, double *est, int *err, hipStream_t s)
{
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_estimate<false>, dim3((unsigned)nq), dim3(EST_BLOCK), 0, s, (const int64_t *)nullptr, q0,
                       set_ptr, set_nodes, sk.n, sk.T, sk.est_scale(), sk.est_q(), sk.node_ptr.ptr, sk.node_samples.ptr,
                       bitmaps, bitmap_words, (uint32_t *)nullptr, (uint64_t)0, cov, est, err);
    SKIS_HIP_TRY(hipGetLastError());
}

void estimate_launch_large(const Sketch &sk, const int64_t *qlist, int64_t g0, int32_t ng, const int64_t *set_ptr,
                           const int32_t *set_nodes, uint32_t *bitmaps, uint64_t bitmap_words, uint32_t *nodebits,
                           unsigned long long *cov, double *est, int *err, hipStream_t s)
{
    if (ng <= 0) return;
    const uint64_t wordsN = ((uint64_t)sk.n + 31) / 32;
    hipLaunchKernelGGL(k_estimate<true>, dim3((unsigned)ng), dim3(EST_BLOCK), 0, s, qlist, g0, set_ptr, set_nodes,
                       sk.n, sk.T, sk.est_scale(), sk.est_q(), sk.node_ptr.ptr, sk.node_samples.ptr, bitmaps, bitmap_words,
                       nodebits, wordsN, cov, est, err);
    SKIS_HIP_TRY(hipGetLastError());
}

void fill_u32(uint32_t *p, uint64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_q<uint32_t>, dim3(gridq(count, 256)), dim3(256), 0, s, count, p, 0u);
    SKIS_HIP_TRY(hipGetLastError());
}

void greedy(const Sketch &sk, QueryScratch &qs, int32_t k, int32_t *seeds, uint64_t *marg, uint64_t *cov_out,
            double *est_out, hipStream_t s)
{
    (void)qs;
    Arena &arena = const_cast<Arena &>(sk.arena);
    const int32_t n = sk.n;
    const uint64_t wordsT = (sk.T + 31) / 32;
    DevBuf<int32_t> delta, delta_spare; // the counts and the buffer a recounting round fills
    DevBuf<uint8_t> chosen;
    DevBuf<uint32_t> covered;
    DevBuf<GreedyState> st;
    const unsigned ga = gridq(((uint64_t)n + ARGMAX_PER - 1) / ARGMAX_PER, 256, 4);
    DevBuf<double> pg;
    DevBuf<int32_t> pv;
    delta.alloc(arena, n);
    delta_spare.alloc(arena, n);
    chosen.alloc(arena, n);
    covered.alloc(arena, wordsT ? wordsT : 1);
    st.alloc(arena, 1);
    pg.alloc(arena, ga);
    pv.alloc(arena, ga);
    hipLaunchKernelGGL(k_greedy_init, dim3(gridq(n, 256)), dim3(256), 0, s, n, sk.node_ptr.ptr, delta.ptr, chosen.ptr);
    hipLaunchKernelGGL(k_fill_q<uint32_t>, dim3(gridq(wordsT ? wordsT : 1, 256)), dim3(256), 0, s,
                       wordsT ? wordsT : 1, covered.ptr, 0u);
    hipLaunchKernelGGL(k_fill_q<int32_t>, dim3(gridq(n, 256)), dim3(256), 0, s, (uint64_t)n, delta_spare.ptr, 0);
    hipLaunchKernelGGL(k_fill_q<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(GreedyState),
                       reinterpret_cast<unsigned char *>(st.ptr), (unsigned char)0);
    SKIS_HIP_TRY(hipGetLastError());
    const unsigned gu = (unsigned)device_cu_count() * 4;
    const int nhot = std::min<int>(sk.nhot, GREEDY_HOT);
    const int32_t *hot_id = nhot > 0 ? sk.hot_id.ptr : nullptr;
    // recount work items (used by the rounds that cover many samples)
    DevBuf<uint32_t> nitems;
    DevBuf<int64_t> ioff;
    DevBuf<RecountItem> items;
    DevBuf<int32_t> work; // the lists cut down by the heavy rounds
    uint64_t nit = 0;
    if (sk.T) {
        nitems.alloc(arena, n);
        ioff.alloc(arena, (size_t)n + 1);
        hipLaunchKernelGGL(k_recount_items_count, dim3(gridq(n, 256)), dim3(256), 0, s, n, sk.node_ptr.ptr,
                           nitems.ptr);
        excl_scan_u32_to_i64(arena, nitems.ptr, ioff.ptr, n, ioff.ptr + n, s);
        int64_t hn = 0;
        SKIS_HIP_TRY(hipMemcpyAsync(&hn, ioff.ptr + n, sizeof(hn), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        nit = (uint64_t)hn;
        items.alloc(arena, nit ? nit : 1);
        work.alloc(arena, sk.entries ? sk.entries : 1);
        hipLaunchKernelGGL(k_recount_items_fill, dim3(gridq(n, 256)), dim3(256), 0, s, n, sk.node_ptr.ptr,
                           nitems.ptr, ioff.ptr, items.ptr);
        SKIS_HIP_TRY(hipGetLastError());
    }
    const unsigned gr = gridq(nit * RECOUNT_LANES, 256, 8);
    for (int32_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(k_greedy_argmax, dim3(ga), dim3(256), 0, s, n, (int)r, sk.T, sk.est_scale(), delta.ptr,
                           delta_spare.ptr, sk.est_q(), chosen.ptr, pg.ptr, pv.ptr, st.ptr, seeds,
                           reinterpret_cast<unsigned long long *>(marg));
        if (sk.T) {
            // the cover lowers delta itself unless the round recounts, decided on the device
            hipLaunchKernelGGL(k_greedy_cover, dim3(gu), dim3(256), 0, s, st.ptr, sk.T, sk.node_ptr.ptr,
                               sk.node_samples.ptr, covered.ptr, sk.sample_ptr.ptr, sk.nodes.ptr, hot_id,
                               sk.hot_node.ptr, nhot, delta.ptr, delta_spare.ptr);
            hipLaunchKernelGGL(k_greedy_recount, dim3(gr), dim3(256), 0, s, st.ptr, sk.T, nit, items.ptr,
                               sk.node_samples.ptr, work.ptr, covered.ptr, delta.ptr, delta_spare.ptr);
        }
    }
    SKIS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_greedy_final, dim3(1), dim3(256), 0, s, k, sk.T, sk.est_scale(), seeds, sk.est_q(), st.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    GreedyState hs;
    SKIS_HIP_TRY(hipMemcpyAsync(&hs, st.ptr, sizeof(hs), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (hs.vstar < 0) throw Error{SKIS_EHIP, "internal error: greedy ran out of candidates"};
    *cov_out = hs.cov;
    *est_out = hs.est;
}

} // namespace skis
