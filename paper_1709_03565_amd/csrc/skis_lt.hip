// skis_lt.hip -- the IIS sampler of the linear threshold model (Sec. 6).
//
// A sample: the root v with probability gamma_v / Gamma (the alias table built over
// gamma_v = sum of v's in-weights), then exactly one in-neighbour of the root, u with
// probability w(u, v) / gamma_v (theta = U * gamma_root against the row's running sums S, the
// first edge with S > theta), then the model's RIS walk: the node added last picks at most one
// in-neighbour, u with probability w(u, x) and none with 1 - sum, until it picks none or a node
// already in the sample.  A node's pick is keyed by (sample id, node) alone, so after the root
// the walk is the orbit x_{k+1} = pick(x_k) of one fixed map: it ends, or it closes on itself.
//
// k_lt_walk: one lane per sample at a time; the walk's nodes sit in the lane's column of LDS
// (at most LT_PATH of them, membership by a scan of the column).  The loop is flattened --
// each iteration moves every lane's walk on by one node or starts the lane's next sample -- so
// that a wave never idles while its longest walk finishes.  Samples that finish in an
// iteration go to staging together: one wave-level prefix sum of their sizes places them in a
// chunk of staging the wave reserved with one atomic.  Walks that outgrow LT_PATH are listed
// for k_lt_long.
//
// k_lt_long: one thread per listed sample and no memory per sample: Brent's cycle finding
// (R. P. Brent, BIT 20, 1980) on the orbit gives the number of distinct nodes before it ends or
// repeats, then the orbit is walked once more to write them.
#include "skis_lt.h"

#include <algorithm>
#include <string>

namespace skis {

constexpr int LT_BLOCK = 256;
constexpr int LT_PATH = 32;              // walk nodes a lane keeps in LDS
constexpr uint32_t LT_WCHUNK = 4096;     // staging entries a wave reserves at a time (> 64 * LT_PATH)
constexpr int LT_LONG_BLOCK = 256;

struct LtCounters {
    unsigned long long stage_used;      // staging entries reserved
    unsigned long long n_long;          // samples listed for k_lt_long
    unsigned long long walk_samples, walk_entries, walk_probed, walk_picks;
    unsigned long long long_entries, long_probed, long_picks;
    int overflow;                       // a reservation ran past the capacity
    int err;                            // 1: a root without in-edges or out of range; 2: a walk past its
                                        // guard; 4: more samples listed for compaction than there are
};

struct LtArgs {
    int32_t n;
    uint32_t count;
    uint64_t j0;
    uint32_t seed_lo, seed_hi;
    uint64_t C;
    const AliasEntry *alias;
    const int32_t *row_ptr;
    const double *S;       // running sums of w along each row
    const double *q;       // 1 - gamma_v
    const uint2 *edges;    // (col, .) per edge
    const uint32_t *wbits; // w bits per edge
    int32_t *staging;
    uint64_t stage_cap;
    uint32_t *out_size;
    unsigned long long *out_off;
    unsigned long long *out_probed;
    int4 *rec;
    uint32_t *long_list;
    uint32_t *medium;
    unsigned long long *n_medium;
    int small_sort;
    LtCounters *ctr;
};

// The first edge e of [lo, hi) with S[e] > theta, hi if there is none (S is nondecreasing
// along a row: its terms w are not negative).
__device__ __forceinline__ int32_t lt_first_above(const double *__restrict__ S, int32_t lo, int32_t hi, double theta)
{
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (S[mid] > theta) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Root of the sample with id (jl, jh) and the in-neighbour it picks (exactly one); deg = the
// root's in-degree.  False for a root outside [0, n) or without in-edges (impossible with a
// valid table: a root has gamma > 0).
__device__ __forceinline__ bool lt_root(const LtArgs &a, uint32_t jl, uint32_t jh, int32_t &root, int32_t &first,
                                        uint32_t &deg)
{
    uint64_t X, Y;
    philox2x64(0u, jl, jh, TAG_ROOT, a.seed_lo, a.seed_hi, X, Y);
    const uint64_t b = __umul64hi(X, (uint64_t)a.n);
    const uint64_t r = __umul64hi(Y, a.C);
    const AliasEntry ae = a.alias[b];
    root = r < ae.thr ? (int32_t)b : ae.alias;
    if (root < 0 || root >= a.n) return false;
    const int32_t rb = a.row_ptr[root], re = a.row_ptr[root + 1];
    if (re <= rb) return false;
    deg = (uint32_t)(re - rb);
    philox2x64(0u, jl, jh, TAG_FIRST, a.seed_lo, a.seed_hi, X, Y);
    const double U = (double)(X >> 11) * 0x1p-53;
    const double theta = __dmul_rn(U, __dsub_rn(1.0, a.q[root]));
    int32_t e = lt_first_above(a.S, rb, re, theta);
    if (e >= re) { // theta rounded up to the row's sum: the last in-edge of positive weight
        e = re - 1;
        while (e > rb && a.wbits[e] == 0u) --e;
    }
    first = (int32_t)a.edges[e].x;
    return true;
}

// The in-neighbour node x picks in the sample with id (jl, jh), -1 for none; deg = x's in-degree.
__device__ __forceinline__ int32_t lt_pick(const LtArgs &a, uint32_t jl, uint32_t jh, int32_t x, uint32_t &deg)
{
    const int32_t rb = a.row_ptr[x], re = a.row_ptr[x + 1];
    uint64_t X, Y;
    philox2x64((uint32_t)x, jl, jh, TAG_LT, a.seed_lo, a.seed_hi, X, Y);
    const double V = (double)(X >> 11) * 0x1p-53;
    deg = (uint32_t)(re - rb);
    const int32_t f = lt_first_above(a.S, rb, re, V);
    return f < re ? (int32_t)a.edges[f].x : -1;
}

__global__ __launch_bounds__(LT_BLOCK) void k_lt_walk(LtArgs a)
{
    __shared__ int32_t s_path[LT_PATH * LT_BLOCK];
    int32_t *const path = s_path + threadIdx.x; // node k of the lane's walk at path[k * LT_BLOCK]
    const uint32_t stride = gridDim.x * LT_BLOCK;
    uint32_t i = blockIdx.x * LT_BLOCK + threadIdx.x; // the lane's current sample
    int len = 0;                                       // nodes of the walk so far (0: start sample i)
    int32_t cur = 0;                                   // the node picked last, not yet checked
    uint32_t jl = 0, jh = 0;
    unsigned long long probed = 0;
    unsigned long long n_fin = 0, n_ent = 0, n_prb = 0, n_picks = 0;
    unsigned long long wpos = 0, wend = 0; // the wave's staging chunk (the same in every lane)
    while (__ballot(i < a.count) != 0ull) {
        bool fin = false;
        if (i < a.count) {
            if (len == 0) {
                const uint64_t j = a.j0 + i;
                jl = (uint32_t)j;
                jh = (uint32_t)(j >> 32);
                int32_t root = 0, first = 0;
                uint32_t deg = 0;
                if (lt_root(a, jl, jh, root, first, deg)) {
                    path[0] = root;
                    len = 1;
                    probed = deg;
                    cur = first;
                    a.rec[i] = make_int4(root, 0, 0, 0);
                } else {
                    atomicOr(&a.ctr->err, 1);
                    path[0] = 0;
                    len = 1;
                    probed = 0;
                    a.rec[i] = make_int4(0, 0, 0, 0);
                    fin = true;
                }
            } else {
                bool seen = false;
                for (int k = 0; k < len; ++k) seen |= path[k * LT_BLOCK] == cur;
                if (seen) {
                    fin = true;
                } else if (len == LT_PATH) {
                    a.long_list[atomicAdd(&a.ctr->n_long, 1ull)] = i;
                    len = 0;
                    i += stride;
                } else {
                    path[len * LT_BLOCK] = cur;
                    ++len;
                    uint32_t deg = 0;
                    const int32_t nx = lt_pick(a, jl, jh, cur, deg);
                    probed += deg;
                    ++n_picks;
                    if (nx < 0) fin = true;
                    else cur = nx;
                }
            }
        }
        // the samples finished in this iteration go to staging together
        const uint32_t need = fin ? (uint32_t)len : 0u;
        const uint32_t incl = wave_incl_scan(need);
        const uint32_t total = lane_value(incl, 63);
        if (total) {
            if (wpos + total > wend) { // the rest of the chunk is left unused
                unsigned long long base = 0;
                if ((threadIdx.x & 63) == 0) base = atomicAdd(&a.ctr->stage_used, (unsigned long long)LT_WCHUNK);
                base = lane_value64(base, 0);
                wpos = base;
                wend = base + LT_WCHUNK;
            }
            if (fin) {
                const unsigned long long off = wpos + incl - need;
                if (off + (unsigned long long)len <= a.stage_cap) {
                    for (int k = 0; k < len; ++k) a.staging[off + k] = path[k * LT_BLOCK];
                } else {
                    atomicOr(&a.ctr->overflow, 1);
                }
                a.out_size[i] = (uint32_t)len;
                a.out_off[i] = off;
                a.out_probed[i] = probed;
                ++n_fin;
                n_ent += (unsigned long long)len;
                n_prb += probed;
                len = 0;
                i += stride;
            }
            wpos += total;
        }
    }
    n_fin = wave_sum(n_fin);
    n_ent = wave_sum(n_ent);
    n_prb = wave_sum(n_prb);
    n_picks = wave_sum(n_picks);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&a.ctr->walk_samples, n_fin);
        atomicAdd(&a.ctr->walk_entries, n_ent);
        atomicAdd(&a.ctr->walk_probed, n_prb);
        atomicAdd(&a.ctr->walk_picks, n_picks);
    }
}

// The number of distinct nodes of the orbit first, pick(first), pick(pick(first)), ... before
// it ends (a pick of none or of the root) or repeats; -1 if the guard trips (it cannot: an orbit
// over n nodes ends or closes within n steps, and Brent's search takes at most a few times that).
__device__ int64_t lt_orbit_length(const LtArgs &a, uint32_t jl, uint32_t jh, int32_t root, int32_t first,
                                   unsigned long long &picks)
{
    const uint64_t guard = 4ull * (uint64_t)a.n + 16;
    uint32_t deg = 0;
    // the cycle length lam: the tortoise waits at x_{2^t - 1} while the hare walks on
    int32_t tort = first, hare = first;
    uint64_t idx = 0, power = 1, lam = 0;
    for (;;) {
        const int32_t nx = lt_pick(a, jl, jh, hare, deg);
        ++picks;
        if (nx < 0 || nx == root) return (int64_t)idx + 1; // the orbit ends after x_idx, all distinct
        hare = nx;
        ++idx;
        ++lam;
        if (hare == tort) break;
        if (lam == power) {
            tort = hare;
            power <<= 1;
            lam = 0;
        }
        if (idx > guard) return -1;
    }
    // the first index mu with x_mu = x_{mu + lam}
    int32_t p = first, r = first;
    for (uint64_t k = 0; k < lam; ++k) {
        r = lt_pick(a, jl, jh, r, deg);
        ++picks;
        if (r < 0) return -1;
    }
    uint64_t mu = 0;
    while (p != r) {
        p = lt_pick(a, jl, jh, p, deg);
        r = lt_pick(a, jl, jh, r, deg);
        picks += 2;
        ++mu;
        if (p < 0 || r < 0 || mu > guard) return -1;
    }
    return (int64_t)(mu + lam);
}

__global__ __launch_bounds__(LT_LONG_BLOCK) void k_lt_long(LtArgs a)
{
    const unsigned long long cnt = a.ctr->n_long;
    unsigned long long n_ent = 0, n_prb = 0, n_picks = 0;
    for (unsigned long long t = (unsigned long long)blockIdx.x * LT_LONG_BLOCK + threadIdx.x; t < cnt;
         t += (unsigned long long)gridDim.x * LT_LONG_BLOCK) {
        const uint32_t i = a.long_list[t];
        const uint64_t j = a.j0 + i;
        const uint32_t jl = (uint32_t)j, jh = (uint32_t)(j >> 32);
        int32_t root = 0, first = 0;
        uint32_t deg = 0;
        int64_t len = -1;
        if (lt_root(a, jl, jh, root, first, deg)) len = lt_orbit_length(a, jl, jh, root, first, n_picks);
        if (len < 0) {
            atomicOr(&a.ctr->err, 2);
            a.out_size[i] = 1;
            a.out_off[i] = 0;
            a.out_probed[i] = 0;
            a.rec[i] = make_int4(0, 0, 0, 0);
            continue;
        }
        const unsigned long long size = 1ull + (unsigned long long)len;
        const unsigned long long off = atomicAdd(&a.ctr->stage_used, size);
        unsigned long long probed = deg;
        if (off + size <= a.stage_cap) {
            a.staging[off] = root;
            int32_t x = first;
            for (int64_t k = 0; k < len; ++k) {
                a.staging[off + 1 + (unsigned long long)k] = x;
                uint32_t dx = 0;
                const int32_t nx = lt_pick(a, jl, jh, x, dx);
                probed += dx;
                ++n_picks;
                x = nx < 0 ? 0 : nx; // the last pick (none, the root or a repeat) is not used
            }
        } else {
            atomicOr(&a.ctr->overflow, 1);
        }
        a.out_size[i] = (uint32_t)size;
        a.out_off[i] = off;
        a.out_probed[i] = probed;
        a.rec[i] = make_int4(root, 0, 0, 0);
        if (size > (unsigned long long)a.small_sort) {
            const unsigned long long k = atomicAdd(a.n_medium, 1ull);
            if (k < a.count) a.medium[k] = i; // bounds guard: report, never index
            else atomicOr(&a.ctr->err, 4);
        }
        n_ent += size;
        n_prb += probed;
    }
    n_ent = wave_sum(n_ent);
    n_prb = wave_sum(n_prb);
    n_picks = wave_sum(n_picks);
    if ((threadIdx.x & 63) == 0 && (n_ent | n_picks)) {
        atomicAdd(&a.ctr->long_entries, n_ent);
        atomicAdd(&a.ctr->long_probed, n_prb);
        atomicAdd(&a.ctr->long_picks, n_picks);
    }
}

// Clears the counters and the compaction's list count before every attempt (a retry after a
// staging overflow lists its samples again).
__global__ void k_lt_zero(LtCounters *c, unsigned long long *n_medium)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *c = LtCounters{};
        *n_medium = 0ull;
    }
}

void sample_lt(Arena &arena, const Prep &prep, int32_t n, const LtIo &io, LtStats &st, hipStream_t s)
{
    if (prep.model != MODEL_LT) throw Error{SKIS_EHIP, "internal error: the LT sampler needs LT preprocessing"};
    if (!prep.alias.ptr || !prep.row_ptr.ptr || !prep.P.ptr || !prep.q.ptr || !prep.edges.ptr || !prep.wbits.ptr ||
        !io.rec || !io.out_size || !io.out_off || !io.out_probed || !io.medium || !io.n_medium || !io.staging)
        throw Error{SKIS_EHIP, "internal error: null buffer for the LT sampler"};
    const uint32_t count = io.count;
    DevBuf<uint32_t> long_list;
    DevBuf<LtCounters> ctr;
    long_list.alloc(arena, count ? count : 1);
    ctr.alloc(arena, 1);
    int blocks_per_cu = 0;
    SKIS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, k_lt_walk, LT_BLOCK, 0));
    if (blocks_per_cu < 1) blocks_per_cu = 1;
    const uint64_t cus = (uint64_t)device_cu_count();
    const uint64_t nblk = std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)blocks_per_cu * cus,
                                                                     ((uint64_t)count + LT_BLOCK - 1) / LT_BLOCK));
    const uint64_t waves = nblk * (LT_BLOCK / 64);
    // every abandoned wave chunk is at least half used (a wave places at most 64 * LT_PATH <
    // LT_WCHUNK / 2 + 1 entries at a time), so 2 * entries + one chunk per wave always fits
    uint64_t cap = io.staging_entries ? io.staging_entries : (uint64_t)count * 8 + waves * LT_WCHUNK + (1u << 20);
    hipEvent_t ev[3];
    for (auto &e : ev) SKIS_HIP_TRY(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 3; ++k) (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    LtCounters hc{};
    for (int attempt = 0;; ++attempt) {
        io.staging->reset();
        io.staging->alloc(arena, cap);
        hipLaunchKernelGGL(k_lt_zero, dim3(1), dim3(64), 0, s, ctr.ptr, io.n_medium);
        LtArgs A{};
        A.n = n;
        A.count = count;
        A.j0 = io.first_id;
        A.seed_lo = io.seed_lo;
        A.seed_hi = io.seed_hi;
        A.C = prep.C;
        A.alias = prep.alias.ptr;
        A.row_ptr = prep.row_ptr.ptr;
        A.S = prep.P.ptr;
        A.q = prep.q.ptr;
        A.edges = prep.edges.ptr;
        A.wbits = prep.wbits.ptr;
        A.staging = io.staging->ptr;
        A.stage_cap = cap;
        A.out_size = io.out_size;
        A.out_off = io.out_off;
        A.out_probed = io.out_probed;
        A.rec = io.rec;
        A.long_list = long_list.ptr;
        A.medium = io.medium;
        A.n_medium = io.n_medium;
        A.small_sort = io.small_sort;
        A.ctr = ctr.ptr;
        if (!A.staging) throw Error{SKIS_EHIP, "internal error: null staging"};
        SKIS_HIP_TRY(hipEventRecord(ev[0], s));
        hipLaunchKernelGGL(k_lt_walk, dim3((unsigned)nblk), dim3(LT_BLOCK), 0, s, A);
        SKIS_HIP_TRY(hipGetLastError());
        SKIS_HIP_TRY(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL(k_lt_long, dim3((unsigned)(cus * 4)), dim3(LT_LONG_BLOCK), 0, s, A);
        SKIS_HIP_TRY(hipGetLastError());
        SKIS_HIP_TRY(hipEventRecord(ev[2], s));
        SKIS_HIP_TRY(hipMemcpyAsync(&hc, ctr.ptr, sizeof(hc), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        if (hc.err)
            throw Error{SKIS_EHIP, "internal error in the LT sampler (flags " + std::to_string(hc.err) + ")"};
        if (!hc.overflow) break;
        if (attempt == 1) throw Error{SKIS_ENOMEM, "LT staging overflow after resize"};
        // every size is known now
        cap = 2 * (hc.walk_entries + hc.long_entries) + waves * LT_WCHUNK + (1u << 20);
    }
    st.walk_samples = hc.walk_samples;
    st.walk_entries = hc.walk_entries;
    st.walk_probed = hc.walk_probed;
    st.walk_picks = hc.walk_picks;
    st.long_samples = hc.n_long;
    st.long_entries = hc.long_entries;
    st.long_probed = hc.long_probed;
    st.long_picks = hc.long_picks;
    if (st.walk_samples + st.long_samples != count)
        throw Error{SKIS_EHIP, "internal error: the LT sampler finished " +
                                   std::to_string(st.walk_samples + st.long_samples) + " of " +
                                   std::to_string(count) + " samples"};
    SKIS_HIP_TRY(hipEventElapsedTime(&st.ms_walk, ev[0], ev[1]));
    SKIS_HIP_TRY(hipEventElapsedTime(&st.ms_long, ev[1], ev[2]));
}

} // namespace skis
