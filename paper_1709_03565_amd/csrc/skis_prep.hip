// skis_prep.hip -- preprocessing for the root draw and the first live in-edge:
// validation, per-row prefix products P and q (Eq. gamma_v / Eq. probn), integer root
// weights W, the weight total C, Gamma (exactly rounded) and the alias table (Eq. probu).
// Under the linear threshold model (Sec. 6) the same kernels form per-row running sums of w
// in place of the products (gamma_v is the sum of v's in-weights).
#include "skis_internal.h"

namespace skis {

enum : int { ERR_ROWPTR = 1, ERR_COL = 2, ERR_SELFLOOP = 4, ERR_WEIGHT = 8, ERR_LTSUM = 16 };

// Linear threshold model: a row's weights may sum to at most 1 (Sec. 6); rounding may take the
// sum past 1 by this much, no more.
constexpr double LT_SUM_SLACK = 0x1p-20;

// q of a row under the linear threshold model from its sum of weights
__device__ __forceinline__ double lt_q(double sum) { return sum < 1.0 ? __dsub_rn(1.0, sum) : 0.0; }

constexpr int32_t LONG_ROW = 256; // rows above this length are taken by a whole workgroup

__device__ __forceinline__ int check_edge(int32_t u, float wf, int64_t v, int32_t n)
{
    int bad = 0;
    if (u < 0 || u >= n) bad |= ERR_COL;
    if (u == (int32_t)v) bad |= ERR_SELFLOOP;
    if (!(wf >= 0.0f && wf <= 1.0f)) bad |= ERR_WEIGHT;
    return bad;
}

// The products of a row (Eq. gamma_v / Eq. probn) are formed left to right:
// P[e] = P[e-1] * (1 - w[e]) with 1 before the row's first edge, one rounding per product
// (the build disables contraction; __dmul_rn / __dsub_rn pin the operations), and
// q[v] = the row's last P (1 for an empty row).  A row's products are one dependent chain
// of multiplies, so a long row is bound by the latency of that chain, not by bandwidth.

// Rows longer than LONG_ROW (with bounds inside [0, m]), listed first so that k_prep_long can
// run beside k_prep_rows.
__global__ __launch_bounds__(256) void k_find_long(int32_t n, int64_t m, const int32_t *__restrict__ row_ptr,
                                                   int32_t *__restrict__ long_rows, unsigned int *__restrict__ n_long)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        if (a >= 0 && (int64_t)b <= m && b - a > LONG_ROW) long_rows[atomicAdd(n_long, 1u)] = (int32_t)v;
    }
}

// One thread per row: validates the row, writes the interleaved (col, w) records, P and q.
// Rows longer than LONG_ROW are k_prep_long's.  lt: running sums S in P (S[e] = S[e-1] + w[e],
// 0 before the row's first edge) and q = 1 - the row's sum.
__global__ __launch_bounds__(256) void k_prep_rows(int32_t n, int64_t m, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const float *__restrict__ w,
                                                   int32_t *__restrict__ rp_copy, uint2 *__restrict__ edges,
                                                   uint32_t *__restrict__ wbits, double *__restrict__ P,
                                                   double *__restrict__ q, int *err, int lt)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        rp_copy[v] = a;
        if (v == n - 1) rp_copy[n] = b;
        int bad = 0;
        if (v == 0 && a != 0) bad |= ERR_ROWPTR;
        if (v == n - 1 && (int64_t)b != m) bad |= ERR_ROWPTR;
        if (a < 0 || (int64_t)b > m || a > b) {
            atomicOr(err, bad | ERR_ROWPTR);
            q[v] = 1.0;
            continue;
        }
        if (b - a > LONG_ROW) { // listed by k_find_long
            if (bad) atomicOr(err, bad);
            continue;
        }
        double run = lt ? 0.0 : 1.0;
        for (int32_t e = a; e < b; ++e) {
            const int32_t u = col[e];
            float wf = w[e];
            bad |= check_edge(u, wf, v, n);
            if (wf == 0.0f) wf = 0.0f; // -0 -> +0: the coin reads the bits
            edges[e] = make_uint2((uint32_t)u, coin_threshold_hi(__float_as_uint(wf)));
            wbits[e] = __float_as_uint(wf);
            run = lt ? __dadd_rn(run, (double)wf) : __dmul_rn(run, __dsub_rn(1.0, (double)wf));
            P[e] = run;
        }
        if (lt) {
            if (run > 1.0 + LT_SUM_SLACK) bad |= ERR_LTSUM;
            q[v] = lt_q(run);
        } else {
            q[v] = run;
        }
        if (bad) atomicOr(err, bad);
    }
}

// One 256-thread workgroup per long row (the next row of the list taken with one atomic, so
// that the workgroup holding the longest row takes no other), LONG_EDGES in-edges at a time,
// every global access coalesced: (1) each thread loads, validates and writes LONG_PER edges and
// puts their factors (1 - w) in LDS (1.0 past the row's end: a multiply by 1 is exact); (2)
// lane 0 carries the row's running product through the chunk, CHAIN_BATCH factors at a time
// held in registers, two register batches in turn: while one batch is multiplied in, the
// other is read from LDS, so that the loop's critical path is the dependent multiplies alone
// and no register copies sit on it; (3) every thread writes its LONG_PER products out.  The
// next chunk's edge loads are in flight during (2).  lt: the terms are w (0 past the row's
// end: adding 0 is exact) and the chain adds.
constexpr int LONG_EDGES = 4096;
constexpr int LONG_PER = LONG_EDGES / 256;
constexpr int CHAIN_BATCH = 16;
static_assert(LONG_EDGES % (2 * CHAIN_BATCH) == 0, "a chunk is whole trips of two batches");

__global__ __launch_bounds__(256) void k_prep_long(int32_t n, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const float *__restrict__ w,
                                                   uint2 *__restrict__ edges, uint32_t *__restrict__ wbits,
                                                   double *__restrict__ P, double *__restrict__ q, int *err,
                                                   const int32_t *__restrict__ long_rows,
                                                   const unsigned int *__restrict__ n_long,
                                                   unsigned int *__restrict__ next_row, int lt)
{
    __shared__ double s_f[LONG_EDGES + CHAIN_BATCH]; // factors of the chunk (+ one batch read ahead)
    __shared__ double s_p[LONG_EDGES];               // their running products
    __shared__ double s_run;
    __shared__ unsigned int s_r;
    const int t = threadIdx.x;
    const unsigned int cnt = *n_long;
    const double ident = lt ? 0.0 : 1.0;
    if (t < CHAIN_BATCH) s_f[LONG_EDGES + t] = ident;
    for (;;) {
        if (t == 0) s_r = atomicAdd(next_row, 1u);
        __syncthreads();
        const unsigned int r = s_r;
        if (r >= cnt) break;
        const int32_t v = long_rows[r];
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        int bad = 0;
        if (t == 0) s_run = ident;
        // element k of a thread's share of a chunk is edge c0 + k * 256 + t (coalesced per k);
        // the loads are unconditional (an index past the row reads its last edge, unused), so
        // that the compiler can keep the next chunk's loads in flight across a chunk
        int32_t uc[LONG_PER];
        float wc[LONG_PER];
#pragma unroll
        for (int k = 0; k < LONG_PER; ++k) {
            const int32_t e = min(a + k * 256 + t, b - 1);
            uc[k] = col[e];
            wc[k] = w[e];
        }
        for (int32_t c0 = a; c0 < b; c0 += LONG_EDGES) {
            // (1) this chunk's edges and factors, then the next chunk's loads
#pragma unroll
            for (int k = 0; k < LONG_PER; ++k) {
                const int32_t e = c0 + k * 256 + t;
                double f = ident;
                if (e < b) {
                    float wf = wc[k];
                    bad |= check_edge(uc[k], wf, v, n);
                    if (wf == 0.0f) wf = 0.0f; // -0 -> +0: the coin reads the bits
                    edges[e] = make_uint2((uint32_t)uc[k], coin_threshold_hi(__float_as_uint(wf)));
                    wbits[e] = __float_as_uint(wf);
                    f = lt ? (double)wf : __dsub_rn(1.0, (double)wf);
                }
                s_f[k * 256 + t] = f;
            }
#pragma unroll
            for (int k = 0; k < LONG_PER; ++k) {
                const int32_t e = min(c0 + LONG_EDGES + k * 256 + t, b - 1);
                uc[k] = col[e];
                wc[k] = w[e];
            }
            __syncthreads();
            const int len = min(b - c0, LONG_EDGES);
            // (2) the chain, in row order
            if (t == 0) {
                // batches i0 .. i0 + 2 CHAIN_BATCH - 1 per trip; entries from len to the end of
                // the trip hold the identity (phase (1) and the read-ahead pad), so running
                // through them leaves the product as it is
                double run = s_run;
                double fa[CHAIN_BATCH], fb[CHAIN_BATCH];
#pragma unroll
                for (int k = 0; k < CHAIN_BATCH; ++k) fa[k] = s_f[k];
                for (int i0 = 0; i0 < len; i0 += 2 * CHAIN_BATCH) {
#pragma unroll
                    for (int k = 0; k < CHAIN_BATCH; ++k) fb[k] = s_f[i0 + CHAIN_BATCH + k];
                    if (lt) {
#pragma unroll
                        for (int k = 0; k < CHAIN_BATCH; ++k) {
                            run = __dadd_rn(run, fa[k]);
                            s_p[i0 + k] = run;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < CHAIN_BATCH; ++k) {
                            run = __dmul_rn(run, fa[k]);
                            s_p[i0 + k] = run;
                        }
                    }
                    // the next trip's first batch (past the chunk: the pad, never used)
                    const int nx = i0 + 2 * CHAIN_BATCH < LONG_EDGES ? i0 + 2 * CHAIN_BATCH : LONG_EDGES;
#pragma unroll
                    for (int k = 0; k < CHAIN_BATCH; ++k) fa[k] = s_f[nx + k];
                    if (lt) {
#pragma unroll
                        for (int k = 0; k < CHAIN_BATCH; ++k) {
                            run = __dadd_rn(run, fb[k]);
                            s_p[i0 + CHAIN_BATCH + k] = run;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < CHAIN_BATCH; ++k) {
                            run = __dmul_rn(run, fb[k]);
                            s_p[i0 + CHAIN_BATCH + k] = run;
                        }
                    }
                }
                s_run = run;
            }
            __syncthreads();
            // (3) the products out (s_f is rewritten by the next chunk's (1) only after every
            // lane has passed the barrier above; s_p by its (2) only after the next barrier)
#pragma unroll
            for (int k = 0; k < LONG_PER; ++k) {
                const int i = k * 256 + t;
                if (i < len) P[c0 + i] = s_p[i];
            }
        }
        __syncthreads();
        if (t == 0) {
            if (lt) {
                if (s_run > 1.0 + LT_SUM_SLACK) bad |= ERR_LTSUM;
                q[v] = lt_q(s_run);
            } else {
                q[v] = s_run;
            }
        }
        if (bad) atomicOr(err, bad);
        __syncthreads();
    }
}

// W_v = ceil(gamma_v * 2^s) and k_v = gamma_v * 2^53 (an integer: gamma_v = 1 - q_v lies on
// the grid 2^-53 Z because q_v is in [0,1]).  Per-block partial sums of W (u64) and k (u128).
__global__ __launch_bounds__(256) void k_weights(int32_t n, int s_shift, const double *__restrict__ q,
                                                 uint64_t *__restrict__ W, uint64_t *__restrict__ partW,
                                                 u128 *__restrict__ partK)
{
    __shared__ uint64_t shW[4];
    __shared__ uint64_t shKlo[4], shKhi[4];
    uint64_t accW = 0;
    u128 accK = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const double g = __dsub_rn(1.0, q[v]);
        const uint64_t k = (uint64_t)ldexp(g, 53);
        uint64_t Wv;
        if (k == 0) {
            Wv = 0;
        } else if (s_shift >= 53) {
            Wv = k << (s_shift - 53);
        } else {
            const int d = 53 - s_shift;
            Wv = (k + ((1ull << d) - 1)) >> d; // ceil(k / 2^d)
        }
        W[v] = Wv;
        accW += Wv;
        accK += (u128)k;
    }
    // block reduction (4 waves)
    accW = wave_sum(accW);
    uint64_t lo = (uint64_t)accK, hi = (uint64_t)(accK >> 64);
    // 128-bit wave sum via two 64-bit halves with carry
    for (int d = 32; d > 0; d >>= 1) {
        uint64_t olo = __shfl_xor(lo, d, 64), ohi = __shfl_xor(hi, d, 64);
        uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1ull : 0ull);
        lo = nlo;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        shW[wid] = accW;
        shKlo[wid] = lo;
        shKhi[wid] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t sw = 0;
        u128 sk = 0;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) {
            sw += shW[i];
            sk += ((u128)shKhi[i] << 64) | shKlo[i];
        }
        partW[blockIdx.x] = sw;
        partK[blockIdx.x] = sk;
    }
}

struct PrepScalars {
    uint64_t C;
    double Gamma;
};

__global__ void k_weights_final(int nb, const uint64_t *partW, const u128 *partK, PrepScalars *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t C = 0;
    u128 K = 0;
    for (int i = 0; i < nb; ++i) {
        C += partW[i];
        K += partK[i];
    }
    out->C = C;
    out->Gamma = ldexp(u128_to_double(K), -53);
}

// ---- alias table: the sequential sweep expressed by prefix sums -------------------------
// Light nodes (a = n*W <= C) in id order have deficits d = C - a, heavy nodes surpluses
// s = a - C.  With inclusive prefix sums D (over lights) and S (over heavies):
//   light i:  thr = a, alias = heavy j with j = min{ j : S_j > D_{i-1} } (itself if none);
//   heavy j:  thr = C + S_j - D_k with k = min{ k : D_k >= S_j }, alias = heavy j+1 (itself
//             for the last heavy, whose thr is then C).
// This reproduces the sweep exactly: the current heavy's remainder after light k is
// C + S_j - D_k, and heavy j turns into a bucket at the first light that brings it to <= C.
__global__ __launch_bounds__(256) void k_alias_flags(int32_t n, const uint64_t *__restrict__ W, uint64_t C,
                                                     uint32_t *__restrict__ light)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        light[v] = ((uint64_t)n * W[v] <= C) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_alias_split(int32_t n, const uint64_t *__restrict__ W, uint64_t C,
                                                     const uint32_t *__restrict__ light,
                                                     const uint32_t *__restrict__ lrank, int32_t *__restrict__ lid,
                                                     int32_t *__restrict__ hid, u128 *__restrict__ dval,
                                                     u128 *__restrict__ sval)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = (uint64_t)n * W[v];
        const uint32_t lr = lrank[v];
        if (light[v]) {
            lid[lr] = (int32_t)v;
            dval[lr] = (u128)(C - a);
        } else {
            const uint32_t hr = (uint32_t)v - lr;
            hid[hr] = (int32_t)v;
            sval[hr] = (u128)(a - C);
        }
    }
}

__global__ __launch_bounds__(256) void k_add_inplace(int64_t len, u128 *__restrict__ excl, const u128 *__restrict__ val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        excl[i] += val[i];
}

__global__ __launch_bounds__(256) void k_alias_light(int32_t n, int64_t L, int64_t H, const uint64_t *__restrict__ W,
                                                     const int32_t *__restrict__ lid, const int32_t *__restrict__ hid,
                                                     const u128 *__restrict__ dval, const u128 *__restrict__ Dinc,
                                                     const u128 *__restrict__ Sinc, AliasEntry *__restrict__ table)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = lid[i];
        const u128 dex = Dinc[i] - dval[i];
        int64_t lo = 0, hi = H; // first j with Sinc[j] > dex
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (Sinc[mid] > dex) hi = mid; else lo = mid + 1;
        }
        AliasEntry e;
        e.thr = (uint64_t)n * W[v];
        e.alias = lo < H ? hid[lo] : v;
        e.pad = 0;
        table[v] = e;
    }
}

__global__ __launch_bounds__(256) void k_alias_heavy(int64_t L, int64_t H, uint64_t C, const int32_t *__restrict__ hid,
                                                     const u128 *__restrict__ Dinc, const u128 *__restrict__ Sinc,
                                                     AliasEntry *__restrict__ table)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < H; j += (int64_t)gridDim.x * blockDim.x) {
        const u128 Sj = Sinc[j];
        int64_t lo = 0, hi = L; // first k with Dinc[k] >= Sj (exists: Sinc[H-1] == Dinc[L-1])
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (Dinc[mid] >= Sj) hi = mid; else lo = mid + 1;
        }
        const int64_t k = lo < L ? lo : L - 1;
        AliasEntry e;
        e.thr = (uint64_t)((u128)C + Sj - Dinc[k]);
        e.alias = j + 1 < H ? hid[j + 1] : hid[j];
        e.pad = 0;
        table[hid[j]] = e;
    }
}

static unsigned grid_for(int64_t items, int block = 256)
{
    int64_t g = (items + block - 1) / block;
    int64_t cap = (int64_t)device_cu_count() * 16;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

static int root_shift(int32_t n)
{
    int L = 0;
    while ((1ll << L) < (int64_t)(n < 2 ? 2 : n)) ++L;
    return 62 - L;
}

void preprocess(Arena &arena, int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                bool build_alias, Prep &out, hipStream_t s, int model)
{
    if (model != MODEL_IC && model != MODEL_LT) throw Error{SKIS_EINVAL, "model must be 0 (IC) or 1 (LT)"};
    out.model = model;
    const int lt = model == MODEL_LT ? 1 : 0;
    out.row_ptr.alloc(arena, (size_t)n + 1);
    const size_t m_quad = (size_t)((m + 3) & ~(int64_t)3);
    out.edges.alloc(arena, m_quad > 0 ? m_quad : 4);
    out.wbits.alloc(arena, (size_t)(m > 0 ? m : 1));
    out.P.alloc(arena, (size_t)(m > 0 ? m : 1));
    out.q.alloc(arena, (size_t)n);
    out.W.alloc(arena, (size_t)n);
    SKIS_HIP_TRY(hipMemsetAsync(out.edges.ptr, 0, out.edges.bytes(), s));
    DevBuf<int> err;
    err.alloc(arena, 4);
    SKIS_HIP_TRY(hipMemsetAsync(err.ptr, 0, 4 * sizeof(int), s));
    DevBuf<int32_t> long_rows;
    long_rows.alloc(arena, (size_t)n);
    unsigned int *n_long = reinterpret_cast<unsigned int *>(err.ptr + 1);
    unsigned int *next_long = reinterpret_cast<unsigned int *>(err.ptr + 2);
    // the long rows' chains (bound by their length) run on a second stream beside the short rows
    hipLaunchKernelGGL(k_find_long, dim3(grid_for(n)), dim3(256), 0, s, n, m, row_ptr, long_rows.ptr, n_long);
    SKIS_HIP_TRY(hipGetLastError());
    hipStream_t s2 = side_stream();
    hipEvent_t fork = nullptr, join = nullptr;
    SKIS_HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *a, *b;
        ~EvGuard()
        {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } evg{&fork, &join};
    SKIS_HIP_TRY(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    SKIS_HIP_TRY(hipEventRecord(fork, s));
    SKIS_HIP_TRY(hipStreamWaitEvent(s2, fork, 0));
    hipLaunchKernelGGL(k_prep_long, dim3((unsigned)device_cu_count() * 4), dim3(256), 0, s2, n, row_ptr, col, w,
                       out.edges.ptr, out.wbits.ptr, out.P.ptr, out.q.ptr, err.ptr, long_rows.ptr, n_long, next_long,
                       lt);
    const hipError_t long_err = hipGetLastError();
    SKIS_HIP_TRY(hipEventRecord(join, s2));
    hipLaunchKernelGGL(k_prep_rows, dim3(grid_for(n)), dim3(256), 0, s, n, m, row_ptr, col, w, out.row_ptr.ptr,
                       out.edges.ptr, out.wbits.ptr, out.P.ptr, out.q.ptr, err.ptr, lt);
    SKIS_HIP_TRY(hipGetLastError());
    SKIS_HIP_TRY(hipStreamWaitEvent(s, join, 0));
    SKIS_HIP_TRY(long_err);
    int herr = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&herr, err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (herr) {
        std::string msg = "invalid graph:";
        if (herr & ERR_ROWPTR) msg += " row_ptr must start at 0, end at m and be nondecreasing;";
        if (herr & ERR_COL) msg += " col entries must lie in [0, n);";
        if (herr & ERR_SELFLOOP) msg += " self-loops are not allowed;";
        if (herr & ERR_WEIGHT) msg += " w must be in [0, 1] (no NaN);";
        if (herr & ERR_LTSUM) msg += " linear threshold model: a node's in-weights must sum to at most 1;";
        throw Error{SKIS_EINVAL, msg};
    }
    const unsigned gw = grid_for(n);
    DevBuf<uint64_t> partW;
    DevBuf<u128> partK;
    DevBuf<PrepScalars> sc;
    partW.alloc(arena, gw);
    partK.alloc(arena, gw);
    sc.alloc(arena, 1);
    hipLaunchKernelGGL(k_weights, dim3(gw), dim3(256), 0, s, n, root_shift(n), out.q.ptr, out.W.ptr, partW.ptr,
                       partK.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_weights_final, dim3(1), dim3(64), 0, s, (int)gw, partW.ptr, partK.ptr, sc.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    PrepScalars hs;
    SKIS_HIP_TRY(hipMemcpyAsync(&hs, sc.ptr, sizeof(hs), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    out.C = hs.C;
    out.Gamma = hs.Gamma;
    if (!build_alias || out.C == 0) return;

    out.alias.alloc(arena, (size_t)n);
    DevBuf<uint32_t> light, lrank, Ltot;
    DevBuf<int32_t> lid, hid;
    DevBuf<u128> dval, sval, Dinc, Sinc;
    light.alloc(arena, n);
    lrank.alloc(arena, n);
    Ltot.alloc(arena, 1);
    lid.alloc(arena, n);
    hid.alloc(arena, n);
    dval.alloc(arena, n);
    sval.alloc(arena, n);
    Dinc.alloc(arena, n);
    Sinc.alloc(arena, n);
    hipLaunchKernelGGL(k_alias_flags, dim3(grid_for(n)), dim3(256), 0, s, n, out.W.ptr, out.C, light.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    excl_scan<uint32_t>(arena, light.ptr, lrank.ptr, n, Ltot.ptr, s);
    uint32_t hL = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&hL, Ltot.ptr, sizeof(hL), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    const int64_t L = hL, H = (int64_t)n - hL;
    hipLaunchKernelGGL(k_alias_split, dim3(grid_for(n)), dim3(256), 0, s, n, out.W.ptr, out.C, light.ptr, lrank.ptr,
                       lid.ptr, hid.ptr, dval.ptr, sval.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    excl_scan<u128>(arena, dval.ptr, Dinc.ptr, L, nullptr, s);
    excl_scan<u128>(arena, sval.ptr, Sinc.ptr, H, nullptr, s);
    hipLaunchKernelGGL(k_add_inplace, dim3(grid_for(L)), dim3(256), 0, s, L, Dinc.ptr, dval.ptr);
    hipLaunchKernelGGL(k_add_inplace, dim3(grid_for(H)), dim3(256), 0, s, H, Sinc.ptr, sval.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_alias_light, dim3(grid_for(L)), dim3(256), 0, s, n, L, H, out.W.ptr, lid.ptr, hid.ptr,
                       dval.ptr, Dinc.ptr, Sinc.ptr, out.alias.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    if (H > 0) {
        hipLaunchKernelGGL(k_alias_heavy, dim3(grid_for(H)), dim3(256), 0, s, L, H, out.C, hid.ptr, Dinc.ptr,
                           Sinc.ptr, out.alias.ptr);
        SKIS_HIP_TRY(hipGetLastError());
    }
    SKIS_HIP_TRY(hipStreamSynchronize(s));
}

} // namespace skis
