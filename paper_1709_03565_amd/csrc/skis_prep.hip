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
constexpr int ROW_BATCH = 8;      // edges a row thread loads at a time

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
// run beside k_prep_rows.  Rows above HUGE_ROW (a few dozen on the largest power-law graphs) are
// listed apart, from the list's far end (long_rows[n - 1 - k]), so that k_prep_long takes them
// first: the longest chain then starts with the kernel instead of wherever the list put it.
// Each workgroup takes a contiguous slice of rows, counts its long rows (LDS atomics), reserves
// their places with one global atomic and lists them in a second pass over the slice: one
// atomic per wave on a single address had cost milliseconds at 40M rows.
constexpr int32_t HUGE_ROW = 1 << 18;
// k_prep_long takes the rows above HUGE_ROW longest first while there are at most this many
// (about 75 on the 1.4B-edge power-law graphs), in list order beyond.
constexpr int HUGE_ORDER_MAX = 1024;

__global__ __launch_bounds__(256) void k_find_long(int32_t n, int64_t m, const int32_t *__restrict__ row_ptr,
                                                   int32_t *__restrict__ long_rows, unsigned int *__restrict__ n_long,
                                                   unsigned int *__restrict__ n_huge)
{
    __shared__ unsigned int s_cnt, s_base, s_cur;
    const int t = threadIdx.x, lane = t & 63;
    const int64_t per = (((int64_t)n + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t v0 = (int64_t)blockIdx.x * per, v1 = v0 + per < (int64_t)n ? v0 + per : (int64_t)n;
    // 0: neither, 1: long, 2: huge
    auto kind = [&](int64_t v) -> int {
        if (v >= v1) return 0;
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        if (!(a >= 0 && (int64_t)b <= m && b - a > LONG_ROW)) return 0;
        return b - a > HUGE_ROW ? 2 : 1;
    };
    if (t == 0) {
        s_cnt = 0;
        s_cur = 0;
    }
    __syncthreads();
    unsigned int mine = 0;
    for (int64_t v = v0 + t; v < v1; v += 256) mine += kind(v) == 1 ? 1u : 0u;
    if (mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (t == 0) s_base = s_cnt ? atomicAdd(n_long, s_cnt) : 0u;
    __syncthreads();
    const unsigned int base = s_base;
    // every lane of a wave runs the same trip count, so the whole wave takes part in each ballot
    for (int64_t v00 = v0; v00 < v1; v00 += 256) {
        const int64_t v = v00 + t;
        const int k = kind(v);
        if (k == 2) long_rows[(int64_t)n - 1 - atomicAdd(n_huge, 1u)] = (int32_t)v;
        const unsigned long long mask = __ballot(k == 1);
        if (mask) {
            unsigned int off = 0;
            if (lane == 0) off = atomicAdd(&s_cur, (unsigned int)__popcll(mask));
            off = (unsigned int)__builtin_amdgcn_readfirstlane((int)off);
            if (k == 1) long_rows[base + off + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)v;
        }
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
        // ROW_BATCH edges at a time, the next batch's loads issued (clamped to the row's last
        // edge, so unconditionally) before this batch is used: one memory latency per batch
        double run = lt ? 0.0 : 1.0;
        if (b > a) {
            int32_t uc[ROW_BATCH];
            float wc[ROW_BATCH];
#pragma unroll
            for (int k = 0; k < ROW_BATCH; ++k) {
                const int32_t e = min(a + k, b - 1);
                uc[k] = col[e];
                wc[k] = w[e];
            }
            for (int32_t e0 = a; e0 < b; e0 += ROW_BATCH) {
                int32_t un[ROW_BATCH];
                float wn[ROW_BATCH];
#pragma unroll
                for (int k = 0; k < ROW_BATCH; ++k) {
                    const int32_t e = min(e0 + ROW_BATCH + k, b - 1);
                    un[k] = col[e];
                    wn[k] = w[e];
                }
#pragma unroll
                for (int k = 0; k < ROW_BATCH; ++k) {
                    const int32_t e = e0 + k;
                    if (e >= b) break;
                    const int32_t u = uc[k];
                    float wf = wc[k];
                    bad |= check_edge(u, wf, v, n);
                    if (wf == 0.0f) wf = 0.0f; // -0 -> +0: the coin reads the bits
                    edges[e] = make_uint2((uint32_t)u, coin_threshold_hi(__float_as_uint(wf)));
                    wbits[e] = __float_as_uint(wf);
                    run = lt ? __dadd_rn(run, (double)wf) : __dmul_rn(run, __dsub_rn(1.0, (double)wf));
                    P[e] = run;
                }
#pragma unroll
                for (int k = 0; k < ROW_BATCH; ++k) {
                    uc[k] = un[k];
                    wc[k] = wn[k];
                }
            }
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
// that the workgroup holding the longest row takes no other; the rows above HUGE_ROW come
// first), LONG_EDGES in-edges at a time.  A row's products are one dependent chain; on the
// longest row that chain bounds the whole preprocessing, so lane 0 of wave 0 does nothing but
// run it: it reads two fp64 factors per LDS read, the reads of the next LONG_TRIP factors in
// flight while the current ones are multiplied (at most nine LDS operations outstanding, so
// the wait for the current factors never waits on the newer reads: with 32 reads in flight
// the 4-bit LDS counter forced a wait for the newest ones), and keeps, every LONG_BLK
// products, the running product before the block (a checkpoint).  The other three waves, at
// the same time, load chunk c + 1 (coalesced, every load of a thread issued before the first
// is used), validate it, write its edge records and w bits and put its factors 1 - w into LDS
// (1 past the row's end: a multiply by 1 leaves the chain as it is), and rebuild the products
// of chunk c - 1: each thread takes a block, starts from its checkpoint and multiplies the
// same factors in the same order, so every product is the chain's own, and writes them out.
// Lane 0 thus issues no store and one LDS read per two factors: a single lane's LDS and global
// stores had made the chain up to four times slower than its multiplies.  Three factor buffers
// rotate (chained, fed, rebuilt).  LT: the terms are w (0 past the row's end) and the chain
// adds.
constexpr int LONG_EDGES = 4096;
constexpr int LONG_TRIP = 16;                  // factors per batch of the chain's LDS reads
constexpr int LONG_PAD = 64;                   // read-ahead past a chunk
constexpr int LONG_BLK = 64;                   // products per checkpoint
constexpr int LONG_FEED = 192;                 // threads of waves 1-3
constexpr int LONG_PER = (LONG_EDGES + LONG_FEED - 1) / LONG_FEED; // edges a feeding thread loads
static_assert(LONG_EDGES % LONG_BLK == 0 && LONG_BLK == 4 * LONG_TRIP, "checkpoints fall on batch quads");
static_assert(LONG_PAD >= LONG_TRIP, "the chain reads one batch past a block");
static_assert(LONG_EDGES / LONG_BLK <= LONG_FEED, "one rebuilt block per feeding thread");

template <bool LT> __device__ __forceinline__ double chain_op(double x, double f)
{
    return LT ? __dadd_rn(x, f) : __dmul_rn(x, f);
}

// Lane 0's chain over one chunk of len factors F (identity terms past len up to the next
// multiple of LONG_BLK plus LONG_TRIP): the checkpoints into CK, the running value returned.
template <bool LT> __device__ __forceinline__ double chain_chunk(const double *F, double *CK, int len, double run)
{
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    double2 xa[LONG_TRIP / 2], xb[LONG_TRIP / 2];
#pragma unroll
    for (int k = 0; k < LONG_TRIP / 2; ++k) xa[k] = F2[k];
    // The empty asm statements pin the order reads -> multiplies -> reads: each takes the
    // running value as an operand (so the multiplies before it stay before it) and orders the
    // LDS reads around it; without them the reads of a batch drift in among the other batch's
    // multiplies and the count of LDS operations in flight passes 15 again.
    for (int i0 = 0; i0 < len; i0 += LONG_BLK) {
        CK[i0 / LONG_BLK] = run; // the product before element i0
        const double2 *B = F2 + i0 / 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int k = 0; k < LONG_TRIP / 2; ++k) xb[k] = B[(2 * h + 1) * (LONG_TRIP / 2) + k];
            asm volatile("" : "+v"(run)::"memory");
#pragma unroll
            for (int k = 0; k < LONG_TRIP / 2; ++k) run = chain_op<LT>(chain_op<LT>(run, xa[k].x), xa[k].y);
            asm volatile("" : "+v"(run)::"memory");
#pragma unroll
            for (int k = 0; k < LONG_TRIP / 2; ++k) xa[k] = B[(2 * h + 2) * (LONG_TRIP / 2) + k];
            asm volatile("" : "+v"(run)::"memory");
#pragma unroll
            for (int k = 0; k < LONG_TRIP / 2; ++k) run = chain_op<LT>(chain_op<LT>(run, xb[k].x), xb[k].y);
            asm volatile("" : "+v"(run)::"memory");
        }
    }
    return run;
}

// A feeding thread's rebuild of block blk of a chunk (len factors F, cnt = min(LONG_BLK,
// len - blk * LONG_BLK) > 0 of them in the block) from its checkpoint x into dst.
template <bool LT>
__device__ __forceinline__ void rebuild_block(const double *F, int blk, int cnt, double x, double *__restrict__ dst)
{
    // two halves of 32 factors (fewer registers: k_prep_rows's waves share the SIMDs)
    const double2 *F2 = reinterpret_cast<const double2 *>(F + blk * LONG_BLK);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double2 f[LONG_BLK / 4];
#pragma unroll
        for (int k = 0; k < LONG_BLK / 4; ++k) f[k] = F2[h * (LONG_BLK / 4) + k];
        double *d = dst + h * (LONG_BLK / 2);
        const int c = cnt - h * (LONG_BLK / 2);
        if (c >= LONG_BLK / 2) {
#pragma unroll
            for (int k = 0; k < LONG_BLK / 4; ++k) {
                x = chain_op<LT>(x, f[k].x);
                d[2 * k] = x;
                x = chain_op<LT>(x, f[k].y);
                d[2 * k + 1] = x;
            }
        } else {
#pragma unroll
            for (int k = 0; k < LONG_BLK / 4; ++k) {
                if (2 * k >= c) break;
                x = chain_op<LT>(x, f[k].x);
                d[2 * k] = x;
                if (2 * k + 1 >= c) break;
                x = chain_op<LT>(x, f[k].y);
                d[2 * k + 1] = x;
            }
        }
    }
}

template <bool LT>
__global__ __launch_bounds__(256) void k_prep_long(int32_t n, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const float *__restrict__ w,
                                                   uint2 *__restrict__ edges, uint32_t *__restrict__ wbits,
                                                   double *__restrict__ P, double *__restrict__ q, int *err,
                                                   const int32_t *__restrict__ long_rows,
                                                   const unsigned int *__restrict__ n_long,
                                                   const unsigned int *__restrict__ n_huge,
                                                   unsigned int *__restrict__ next_row)
{
    __shared__ __align__(16) double s_f[3][LONG_EDGES + LONG_PAD]; // factors of three chunks (+ read-ahead pad)
    __shared__ double s_ck[2][LONG_EDGES / LONG_BLK];               // checkpoints of two chunks
    __shared__ int32_t s_hrow[HUGE_ORDER_MAX], s_hlen[HUGE_ORDER_MAX];
    __shared__ unsigned int s_r;
    __shared__ int32_t s_pick;
    const int t = threadIdx.x;
    const unsigned int nh = *n_huge, cnt = nh + *n_long;
    const double ident = LT ? 0.0 : 1.0;
    for (int i = t; i < LONG_PAD; i += 256) s_f[0][LONG_EDGES + i] = s_f[1][LONG_EDGES + i] = s_f[2][LONG_EDGES + i] = ident;
    // waves 1-3 put chunk c0 of row v (edges [c0, b)) into buffer `buf`; returns their flags.
    // Every load and store is unconditional, at the edge clamped to the row's last one (a
    // clamped store writes the value that edge's own thread writes), so the compiler's wait
    // counts stay exact: with loads and stores under branches it waited for every store.
    auto feed = [&](int32_t v, int32_t c0, int32_t b, int buf) -> int {
        int32_t u[LONG_PER];
        float wf[LONG_PER];
#pragma unroll
        for (int k = 0; k < LONG_PER; ++k) {
            const int32_t ec = min(c0 + t - 64 + k * LONG_FEED, b - 1);
            u[k] = col[ec];
            wf[k] = w[ec];
        }
        int bad = 0;
#pragma unroll
        for (int k = 0; k < LONG_PER; ++k) {
            const int i = t - 64 + k * LONG_FEED;
            const int32_t e = c0 + i, ec = min(e, b - 1);
            float x = wf[k];
            bad |= check_edge(u[k], x, v, n);
            if (x == 0.0f) x = 0.0f; // -0 -> +0: the coin reads the bits
            edges[ec] = make_uint2((uint32_t)u[k], coin_threshold_hi(__float_as_uint(x)));
            wbits[ec] = __float_as_uint(x);
            const double f = e < b ? (LT ? (double)x : __dsub_rn(1.0, (double)x)) : ident;
            if (k + 1 < LONG_PER || i < LONG_EDGES) s_f[buf][i] = f;
        }
        return bad;
    };
    for (;;) {
        if (t == 0) s_r = atomicAdd(next_row, 1u);
        __syncthreads();
        const unsigned int r = s_r;
        if (r >= cnt) break;
        int32_t v;
        if (r >= nh) {
            v = long_rows[r - nh];
        } else if (nh > (unsigned int)HUGE_ORDER_MAX) {
            v = long_rows[(int64_t)n - 1 - r];
        } else {
            // place r of the huge rows by length, longest first (equal lengths by row id): the
            // row that exactly r rows go before
            for (unsigned int j = t; j < nh; j += 256) {
                const int32_t x = long_rows[(int64_t)n - 1 - j];
                s_hrow[j] = x;
                s_hlen[j] = row_ptr[x + 1] - row_ptr[x];
            }
            __syncthreads();
            for (unsigned int j = t; j < nh; j += 256) {
                const int32_t lj = s_hlen[j], vj = s_hrow[j];
                unsigned int rank = 0;
                for (unsigned int i = 0; i < nh; ++i)
                    rank += (s_hlen[i] > lj || (s_hlen[i] == lj && s_hrow[i] < vj)) ? 1u : 0u;
                if (rank == r) s_pick = vj;
            }
            __syncthreads();
            v = s_pick;
        }
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        const int nchunks = (b - a + LONG_EDGES - 1) / LONG_EDGES;
        int bad = 0;
        if (t >= 64) bad |= feed(v, a, b, 0);
        __syncthreads();
        double run = ident; // lane 0's chain
        for (int c = 0; c <= nchunks; ++c) {
            if (t == 0) {
                if (c < nchunks)
                    run = chain_chunk<LT>(s_f[c % 3], s_ck[c & 1], min(b - (a + c * LONG_EDGES), LONG_EDGES), run);
            } else if (t >= 64) {
                if (c + 1 < nchunks) bad |= feed(v, a + (c + 1) * LONG_EDGES, b, (c + 1) % 3);
                if (c >= 1) { // rebuild chunk c - 1 from its checkpoints, one block per thread
                    const int32_t cp0 = a + (c - 1) * LONG_EDGES;
                    const int lenp = min(b - cp0, LONG_EDGES);
                    const int blk = t - 64;
                    if (blk * LONG_BLK < lenp)
                        rebuild_block<LT>(s_f[(c - 1) % 3], blk, min(LONG_BLK, lenp - blk * LONG_BLK),
                                          s_ck[(c - 1) & 1][blk], P + cp0 + blk * LONG_BLK);
                }
            }
            __syncthreads();
        }
        if (t == 0) {
            if (LT) {
                if (run > 1.0 + LT_SUM_SLACK) bad |= ERR_LTSUM;
                q[v] = lt_q(run);
            } else {
                q[v] = run;
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

// k_prep_rows's grid: at most as many workgroups per CU as leave one k_prep_long wave room in
// every SIMD's registers beside them (512 VGPRs a lane, allocated in steps of 8; at most 8 waves
// a SIMD), so that the long rows' chains start with their kernel whichever of the two kernels
// the device starts first (filling every CU, k_prep_rows had held the longest chain back by
// about 19 ms at 40M rows).  A k_prep_rows workgroup puts one wave on each SIMD.
static unsigned prep_rows_grid(int64_t n)
{
    auto vgprs = [](const void *fn) {
        hipFuncAttributes a{};
        if (hipFuncGetAttributes(&a, fn) != hipSuccess || a.numRegs <= 0) return 256;
        return (a.numRegs + 7) / 8 * 8;
    };
    const int vr = vgprs(reinterpret_cast<const void *>(k_prep_rows));
    const int vl = std::max(vgprs(reinterpret_cast<const void *>(k_prep_long<false>)),
                            vgprs(reinterpret_cast<const void *>(k_prep_long<true>)));
    const int per_simd = std::max(1, std::min(7, (512 - vl) / vr));
    const int64_t cap = (int64_t)device_cu_count() * per_simd;
    const int64_t g = std::min<int64_t>((n + 255) / 256, cap);
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
    // every edge record below m is written by the row kernels; the quad padding past m is clear
    if (out.edges.count > (size_t)m)
        SKIS_HIP_TRY(hipMemsetAsync(out.edges.ptr + m, 0, (out.edges.count - (size_t)m) * sizeof(uint2), s));
    DevBuf<int> err;
    err.alloc(arena, 4);
    SKIS_HIP_TRY(hipMemsetAsync(err.ptr, 0, 4 * sizeof(int), s));
    DevBuf<int32_t> long_rows;
    long_rows.alloc(arena, (size_t)n);
    unsigned int *n_long = reinterpret_cast<unsigned int *>(err.ptr + 1);
    unsigned int *next_long = reinterpret_cast<unsigned int *>(err.ptr + 2);
    unsigned int *n_huge = reinterpret_cast<unsigned int *>(err.ptr + 3);
    if (reinterpret_cast<uintptr_t>(out.P.ptr) & 15) throw Error{SKIS_EHIP, "internal error: P is not 16-byte aligned"};
    // The long rows' chains (bound by their length) run beside the short rows.  k_prep_long
    // follows k_find_long on the caller's stream and k_prep_rows goes to a second stream, which
    // first waits for the listing: the device then starts the chains first (when k_prep_rows
    // was dispatched first, the other stream's kernels started milliseconds late, and the
    // longest chain with them).
    hipLaunchKernelGGL(k_find_long, dim3(grid_for(n)), dim3(256), 0, s, n, m, row_ptr, long_rows.ptr, n_long, n_huge);
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
    hipLaunchKernelGGL(lt ? k_prep_long<true> : k_prep_long<false>, dim3((unsigned)device_cu_count()), dim3(256), 0, s,
                       n, row_ptr, col, w, out.edges.ptr, out.wbits.ptr, out.P.ptr, out.q.ptr, err.ptr, long_rows.ptr,
                       n_long, n_huge, next_long);
    const hipError_t long_err = hipGetLastError();
    // from here on, s waits for s2 before anything else, whatever fails
    hipError_t side_err = hipStreamWaitEvent(s2, fork, 0);
    if (side_err == hipSuccess) {
        hipLaunchKernelGGL(k_prep_rows, dim3(prep_rows_grid(n)), dim3(256), 0, s2, n, m, row_ptr, col, w,
                           out.row_ptr.ptr, out.edges.ptr, out.wbits.ptr, out.P.ptr, out.q.ptr, err.ptr, lt);
        side_err = hipGetLastError();
    }
    const hipError_t rec_err = hipEventRecord(join, s2);
    if (rec_err != hipSuccess) (void)hipStreamSynchronize(s2); // no event to wait on: drain it here
    SKIS_HIP_TRY(rec_err);
    SKIS_HIP_TRY(hipStreamWaitEvent(s, join, 0));
    SKIS_HIP_TRY(long_err);
    SKIS_HIP_TRY(side_err);
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
