/*
 * skis_oracle.c -- plain, slow CPU oracle for the SKIS hot path (Nguyen, Thai, Dinh,
 * "Importance Sketching of Influence Dynamics in Billion-scale Networks", ICDM 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no source with the HIP path: Philox, the prefix products, the alias table,
 * the sampler, the compaction, the coverage counter and the greedy are all written
 * again here, as directly as the paper states them.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread.
 * Every floating-point value that decides an integer (prefix products P, the bucket
 * threshold, the greedy gains) is computed in IEEE binary64 in the order written here.
 *
 * Canonical randomness map (the paper draws coins but fixes no generator):
 *   Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11), key = 64-bit seed,
 *   counter = (sub, j_lo, j_hi, tag) for sample id j.
 *     tag 0 (root draw):       sub = 0; X = y1:y0 picks the alias bucket, Y = y3:y2 its split
 *     tag 1 (first live edge): sub = 0; U = (X >> 11) * 2^-53
 *     tag 2 (edge coin, high): sub = e >> 2; word y[e & 3] is the high half of edge e's coin
 *     tag 3 (edge coin, low):  sub = e;      word y0 is the low half of edge e's coin
 *                              the coin is the 64-bit word high:low; the edge is live iff
 *                              w >= 1 or coin < floor(w * 2^64)
 *     tag 4 (LT selection):    sub = x;      U = (X >> 11) * 2^-53 picks node x's in-neighbour in
 *                              the linear threshold model (none when U >= the row's weight sum)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ENOMEM (-2)
#define ORA_WDEGENERATE 1

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplications,
 * the key bumped by the Weyl constants between rounds.
 * ---------------------------------------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The two 64-bit halves of one Philox call for (sub, j, tag). */
static void draw2(uint64_t seed, uint32_t sub, uint64_t j, uint32_t tag, uint64_t *X, uint64_t *Y)
{
    uint32_t ctr[4] = {sub, (uint32_t)j, (uint32_t)(j >> 32), tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t y[4];
    ora_philox4x32_10(ctr, key, y);
    *X = ((uint64_t)y[1] << 32) | y[0];
    *Y = ((uint64_t)y[3] << 32) | y[2];
}

static uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

/* Live-edge coin of edge e in sample j (Sec. 2.1: each edge is live independently with
 * probability w).  The coin is the 64-bit word high:low drawn as the randomness map above
 * states; floor(w * 2^64) is exact for every fp32 w >= 2^-40, so the coin is live with
 * probability exactly w there.  Two 64-bit words compare as their (high, low) pairs do
 * lexicographically, so the low half is only drawn when the high halves are equal. */
int ora_edge_coin(uint64_t seed, uint64_t j, int64_t e, float w)
{
    if (w >= 1.0f) return 1;
    const uint64_t thr = (uint64_t)((double)w * 0x1p64);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t y[4];
    const uint32_t hi_ctr[4] = {(uint32_t)((uint64_t)e >> 2), (uint32_t)j, (uint32_t)(j >> 32), 2u};
    ora_philox4x32_10(hi_ctr, key, y);
    const uint32_t hi = y[e & 3], thr_hi = (uint32_t)(thr >> 32);
    if (hi != thr_hi) return hi < thr_hi;
    const uint32_t lo_ctr[4] = {(uint32_t)e, (uint32_t)j, (uint32_t)(j >> 32), 3u};
    ora_philox4x32_10(lo_ctr, key, y);
    return y[0] < (uint32_t)thr;
}

/* ------------------------------------------------------------------------------------
 * Input validation (problem statement, Sec. 2: w(u,v) in [0,1]; plus the canonical
 * in-CSR contract).  Returns ORA_OK or ORA_EINVAL.
 * ---------------------------------------------------------------------------------- */
int ora_validate(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w)
{
    if (n <= 0 || m < 0 || m > INT32_MAX) return ORA_EINVAL;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != m) return ORA_EINVAL;
    for (int32_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] < row_ptr[v]) return ORA_EINVAL;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n || col[e] == v) return ORA_EINVAL;
            if (!(w[e] >= 0.0f && w[e] <= 1.0f)) return ORA_EINVAL; /* also rejects NaN */
        }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------------------
 * Eq. (gamma_v) and the bucket probabilities of Eq. (probn): per row v, the product P_e
 * of (1 - w) over the in-edges up to and including e, in CSR order.  q_v = P of the last
 * in-edge (1 for an empty row) is the singular probability, and gamma_v = 1 - q_v.
 * The paper defines these products over the reals; in binary64 they are formed left to
 * right, P_e = P_{e-1} * (1 - w_e) with P before the row's first edge equal to 1, one
 * rounding per product.
 * ---------------------------------------------------------------------------------- */
void ora_row_prefix(int32_t n, const int32_t *row_ptr, const float *w, double *P, double *q)
{
    for (int32_t v = 0; v < n; ++v) {
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        double run = 1.0;
        for (int32_t e = a; e < b; ++e) {
            run = run * (1.0 - (double)w[e]);
            P[e] = run;
        }
        q[v] = run;
    }
}

/* The linear threshold model (Sec. 6): node v picks at most one in-neighbour, u with probability
 * w(u,v), none with probability 1 - sum_u w(u,v), so gamma_v = sum_u w(u,v) (the weights of a
 * row must sum to at most 1).  Per row, S_e = S_{e-1} + w_e left to right in binary64 (S before
 * the first edge is 0), and q_v = 1 - S of the last edge (1 for an empty row), 0 if the sum
 * exceeds 1 by rounding.  Returns ORA_EINVAL if a row's sum exceeds 1 + 2^-20. */
int ora_row_sums_lt(int32_t n, const int32_t *row_ptr, const float *w, double *S, double *q)
{
    int st = ORA_OK;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t a = row_ptr[v], b = row_ptr[v + 1];
        double run = 0.0;
        for (int32_t e = a; e < b; ++e) {
            run = run + (double)w[e];
            S[e] = run;
        }
        if (run > 1.0 + 0x1p-20) st = ORA_EINVAL;
        q[v] = run < 1.0 ? 1.0 - run : 0.0;
    }
    return st;
}

/* Gamma = sum_v gamma_v (Table 1), rounded once.  Each gamma_v = 1 - q_v with q_v in
 * [0,1] lies on the grid 2^-53 Z, so the sum is exact in a 128-bit integer. */
double ora_gamma_total(int32_t n, const double *q)
{
    unsigned __int128 acc = 0;
    for (int32_t v = 0; v < n; ++v) {
        double g = 1.0 - q[v];
        double k = ldexp(g, 53);
        acc += (unsigned __int128)(uint64_t)k;
    }
    return ldexp((double)acc, -53);
}

/* Integer root weights for Eq. (probu): W_v = ceil(gamma_v * 2^s), s = 62 - ceil(log2 n),
 * so that P(root = v) = W_v / C with C = sum W_v, and W_v > 0 exactly when gamma_v > 0. */
int ora_root_shift(int32_t n)
{
    int L = 0;
    while (((int64_t)1 << L) < (int64_t)(n < 2 ? 2 : n)) ++L;
    return 62 - L;
}

uint64_t ora_root_weights(int32_t n, const double *q, uint64_t *W)
{
    int s = ora_root_shift(n);
    uint64_t C = 0;
    for (int32_t v = 0; v < n; ++v) {
        double g = 1.0 - q[v];
        W[v] = g > 0.0 ? (uint64_t)ceil(ldexp(g, s)) : 0u;
        C += W[v];
    }
    return C;
}

/* ------------------------------------------------------------------------------------
 * Alias table for the root draw (Eq. probu), Walker/Vose style, built by one sequential
 * sweep.  Node v owns a_v = n * W_v units of mass; each of the n buckets holds C units.
 * Light nodes (a_v <= C) in ascending id order are filled from the current heavy node
 * (the first, in ascending id order, with mass left over); a heavy node whose remainder
 * drops to <= C becomes a bucket in its own right at once, filled from the next heavy.
 * Bucket b: with r uniform in [0, C), the draw is b if r < thr[b], else alias[b].
 * ---------------------------------------------------------------------------------- */
int ora_alias_build(int32_t n, const uint64_t *W, uint64_t C, uint64_t *thr, int32_t *alias)
{
    int32_t *light = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *heavy = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!light || !heavy) { free(light); free(heavy); return ORA_ENOMEM; }
    int32_t nl = 0, nh = 0;
    for (int32_t v = 0; v < n; ++v) {
        uint64_t a = (uint64_t)n * W[v];
        if (a <= C) light[nl++] = v; else heavy[nh++] = v;
    }
    int32_t j = 0;
    uint64_t res = nh > 0 ? (uint64_t)n * W[heavy[0]] : 0;
    for (int32_t i = 0; i < nl; ++i) {
        int32_t l = light[i];
        uint64_t a = (uint64_t)n * W[l];
        thr[l] = a;
        if (j < nh) {
            alias[l] = heavy[j];
            res -= (C - a);
        } else {
            alias[l] = l; /* only when a == C: every unit of surplus is already placed */
        }
        while (j < nh && res <= C) {
            int32_t h = heavy[j];
            thr[h] = res;
            if (j + 1 < nh) {
                alias[h] = heavy[j + 1];
                res = (uint64_t)n * W[heavy[j + 1]] - (C - res);
            } else {
                alias[h] = h;
            }
            ++j;
        }
    }
    free(light);
    free(heavy);
    return ORA_OK;
}

/* ------------------------------------------------------------------------------------
 * One IIS sample (Alg. 1) under the canonical randomness map.
 * Graph, prefix products and alias table are shared read-only; `mark` is a zeroed
 * byte array of n entries owned by the caller and zeroed again on return.
 * Writes R_j (sorted ascending) into *buf (grown with realloc), returns |R_j|.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col;
    const float *w;
    const double *P, *q;
    const uint64_t *thr;
    const int32_t *alias;
    uint64_t C;
    uint64_t seed;
    int ris_mode; /* 1: plain RIS sample (uniform root, no conditioning), Sec. 2.3.1 */
    int model;    /* 0: independent cascade; 1: linear threshold (P holds the row sums S) */
} ora_ctx;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    int32_t *nodes;
    int64_t len, cap;
} ora_vec;

static int vec_push(ora_vec *v, int32_t x)
{
    if (v->len == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 1024;
        int32_t *p = (int32_t *)realloc(v->nodes, sizeof(int32_t) * (size_t)nc);
        if (!p) return ORA_ENOMEM;
        v->nodes = p;
        v->cap = nc;
    }
    v->nodes[v->len++] = x;
    return ORA_OK;
}

/* Appends R_j to out (sorted); returns its size, or a negative error code. */
static int64_t ora_one_sample(const ora_ctx *g, uint64_t j, unsigned char *mark, ora_vec *out,
                              int32_t *root_out, uint64_t *probed_out)
{
    const int64_t base = out->len;
    uint64_t X, Y;
    int32_t root;

    /* Alg. 1, the root: drawn with probability gamma_v / Gamma (Eq. probu), by the alias
     * table over integer weights; in RIS mode a uniform root (Sec. 2.3.1 step 1). */
    draw2(g->seed, 0u, j, 0u, &X, &Y);
    uint64_t b = mulhi64(X, (uint64_t)g->n);
    if (g->ris_mode) {
        root = (int32_t)b;
    } else {
        uint64_t r = mulhi64(Y, g->C);
        root = r < g->thr[b] ? (int32_t)b : g->alias[b];
    }
    if (vec_push(out, root)) return ORA_ENOMEM;
    mark[root] = 1;

    const int32_t rs = g->row_ptr[root], re = g->row_ptr[root + 1];
    int32_t first_scan = rs; /* first in-edge of the root that still gets a coin */
    if (!g->ris_mode) {
        /* Alg. 1, the first live in-edge, Eq. (probn): bucket B_i has probability
         * prod_{t<i}(1-w_t) w_i / gamma = (P_{i-1} - P_i) / gamma.  With theta uniform in
         * [0, gamma), B_i is the first i whose cumulative mass 1 - P_i exceeds theta. */
        draw2(g->seed, 0u, j, 1u, &X, &Y);
        double U = (double)(X >> 11) * 0x1p-53;
        double gamma_root = 1.0 - g->q[root];
        double theta = U * gamma_root;
        int32_t istar = -1;
        for (int32_t e = rs; e < re; ++e) {
            if (1.0 - g->P[e] > theta) { istar = e; break; }
        }
        if (istar < 0) { /* theta rounded up to gamma: take the last bucket of positive mass */
            for (int32_t e = re - 1; e >= rs; --e)
                if (g->w[e] > 0.0f) { istar = e; break; }
        }
        /* Alg. 1: u_i joins R_j and the queue. */
        int32_t u = g->col[istar];
        if (!mark[u]) {
            mark[u] = 1;
            if (vec_push(out, u)) return ORA_ENOMEM;
        }
        /* Alg. 1, the root's other in-edges, with the bucket reading: in-edges before u_i are dead (that is
         * what B_i means), in-edges after it flip their own coins. */
        first_scan = istar + 1;
    }
    for (int32_t e = first_scan; e < re; ++e) {
        int32_t u = g->col[e];
        if (!mark[u] && ora_edge_coin(g->seed, j, e, g->w[e])) {
            mark[u] = 1;
            if (vec_push(out, u)) return ORA_ENOMEM;
        }
    }
    /* Alg. 1, the FIFO reverse BFS; the root itself is not queued again. */
    for (int64_t head = base + 1; head < out->len; ++head) {
        int32_t x = out->nodes[head];
        for (int32_t e = g->row_ptr[x]; e < g->row_ptr[x + 1]; ++e) {
            int32_t u = g->col[e];
            if (!mark[u] && ora_edge_coin(g->seed, j, e, g->w[e])) {
                mark[u] = 1;
                if (vec_push(out, u)) return ORA_ENOMEM;
            }
        }
    }
    uint64_t probed = 0;
    for (int64_t i = base; i < out->len; ++i) {
        int32_t x = out->nodes[i];
        probed += (uint64_t)(g->row_ptr[x + 1] - g->row_ptr[x]);
        mark[x] = 0;
    }
    int64_t size = out->len - base;
    qsort(out->nodes + base, (size_t)size, sizeof(int32_t), cmp_i32);
    *root_out = root;
    *probed_out = probed;
    return size;
}

/* The first in-edge e of [a, b) with S_e > theta, or b if there is none. */
static int32_t ora_first_above(const double *S, int32_t a, int32_t b, double theta)
{
    for (int32_t e = a; e < b; ++e)
        if (S[e] > theta) return e;
    return b;
}

/* One IIS sample under the linear threshold model (Sec. 6): the root as in Alg. 1 (weights
 * gamma_v / Gamma), exactly one of its in-neighbours, u with probability w(u, root) / gamma_root
 * (theta = U * gamma_root against the row sums), then the RIS walk of the model: the last node
 * added picks at most one in-neighbour (tag-4 draw of that node), until it picks none or picks a
 * node already in the sample.  Appends R_j (sorted) to out; returns its size. */
static int64_t ora_one_sample_lt(const ora_ctx *g, uint64_t j, unsigned char *mark, ora_vec *out,
                                 int32_t *root_out, uint64_t *probed_out)
{
    const int64_t base = out->len;
    uint64_t X, Y;
    draw2(g->seed, 0u, j, 0u, &X, &Y);
    const uint64_t b = mulhi64(X, (uint64_t)g->n);
    const uint64_t r = mulhi64(Y, g->C);
    const int32_t root = r < g->thr[b] ? (int32_t)b : g->alias[b];
    if (vec_push(out, root)) return ORA_ENOMEM;
    mark[root] = 1;
    const int32_t rs = g->row_ptr[root], re = g->row_ptr[root + 1];
    draw2(g->seed, 0u, j, 1u, &X, &Y);
    const double U = (double)(X >> 11) * 0x1p-53;
    const double theta = U * (1.0 - g->q[root]);
    int32_t e = ora_first_above(g->P, rs, re, theta);
    if (e >= re) { /* theta rounded up to the row's sum: the last in-edge of positive weight */
        for (e = re - 1; e > rs && g->w[e] <= 0.0f; --e) {
        }
    }
    int32_t x = g->col[e];
    while (!mark[x]) {
        mark[x] = 1;
        if (vec_push(out, x)) return ORA_ENOMEM;
        draw2(g->seed, (uint32_t)x, j, 4u, &X, &Y);
        const double V = (double)(X >> 11) * 0x1p-53;
        const int32_t xs = g->row_ptr[x], xe = g->row_ptr[x + 1];
        const int32_t f = ora_first_above(g->P, xs, xe, V);
        if (f >= xe) break; /* x picks no in-neighbour */
        x = g->col[f];
    }
    uint64_t probed = 0;
    for (int64_t i = base; i < out->len; ++i) {
        const int32_t y = out->nodes[i];
        probed += (uint64_t)(g->row_ptr[y + 1] - g->row_ptr[y]);
        mark[y] = 0;
    }
    const int64_t size = out->len - base;
    qsort(out->nodes + base, (size_t)size, sizeof(int32_t), cmp_i32);
    *root_out = root;
    *probed_out = probed;
    return size;
}

/* ------------------------------------------------------------------------------------
 * A sketch over sample ids [j0, j1): Alg. 2's preprocessing, kept as a CSR hypergraph.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    uint64_t j0, j1;
    int64_t entries;
    uint64_t probed_total;
    int64_t *sample_ptr; /* [count + 1] */
    int32_t *nodes;      /* [entries] */
    int32_t *roots;      /* [count] */
    uint64_t *probed;    /* [count] */
    double Gamma;
    uint64_t C;
    int status;
} ora_sketch;

typedef struct {
    const ora_ctx *g;
    uint64_t j0, j1;
    ora_vec out;
    int64_t *sizes;
    int32_t *roots;
    uint64_t *probed;
    int status;
} ora_worker;

static void *ora_worker_run(void *arg)
{
    ora_worker *wk = (ora_worker *)arg;
    unsigned char *mark = (unsigned char *)calloc((size_t)wk->g->n, 1);
    if (!mark) { wk->status = ORA_ENOMEM; return NULL; }
    for (uint64_t j = wk->j0; j < wk->j1; ++j) {
        int32_t root;
        uint64_t probed;
        int64_t s = wk->g->model == 1 ? ora_one_sample_lt(wk->g, j, mark, &wk->out, &root, &probed)
                                      : ora_one_sample(wk->g, j, mark, &wk->out, &root, &probed);
        if (s < 0) { wk->status = (int)s; break; }
        wk->sizes[j - wk->j0] = s;
        wk->roots[j - wk->j0] = root;
        wk->probed[j - wk->j0] = probed;
    }
    free(mark);
    return NULL;
}

void ora_sketch_free(ora_sketch *s)
{
    if (!s) return;
    free(s->sample_ptr);
    free(s->nodes);
    free(s->roots);
    free(s->probed);
    free(s);
}

/* ------------------------------------------------------------------------------------
 * Alg. 2's preprocessing, done once per graph: validation, the prefix products P and q
 * (Eq. gamma_v), Gamma, the integer root weights and the alias table (Eq. probu).  The
 * graph arrays are borrowed and must outlive the object.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *row_ptr, *col;
    const float *w;
    double *P, *q;
    uint64_t *W, *thr;
    int32_t *alias;
    double Gamma;
    uint64_t C;
    int model;  /* 0: independent cascade (P = prefix products); 1: linear threshold (P = row sums) */
    int status; /* ORA_OK, ORA_WDEGENERATE (Gamma = 0) or a negative error */
} ora_prep;

void ora_prep_free(ora_prep *p)
{
    if (!p) return;
    free(p->P); free(p->q); free(p->W); free(p->thr); free(p->alias);
    free(p);
}

ora_prep *ora_prepare_model(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                            int model)
{
    ora_prep *p = (ora_prep *)calloc(1, sizeof(ora_prep));
    if (!p) return NULL;
    p->n = n; p->m = m; p->row_ptr = row_ptr; p->col = col; p->w = w; p->model = model;
    p->status = ora_validate(n, m, row_ptr, col, w);
    if (!p->status && (model < 0 || model > 1)) p->status = ORA_EINVAL;
    if (p->status) return p;
    p->P = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    p->q = (double *)malloc(sizeof(double) * (size_t)n);
    p->W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    p->thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    p->alias = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!p->P || !p->q || !p->W || !p->thr || !p->alias) { p->status = ORA_ENOMEM; return p; }
    if (model == 1) {
        p->status = ora_row_sums_lt(n, row_ptr, w, p->P, p->q);
        if (p->status) return p;
    } else {
        ora_row_prefix(n, row_ptr, w, p->P, p->q);
    }
    p->Gamma = ora_gamma_total(n, p->q);
    p->C = ora_root_weights(n, p->q, p->W);
    if (p->C == 0) { p->status = ORA_WDEGENERATE; return p; } /* no non-singular sample exists */
    if (ora_alias_build(n, p->W, p->C, p->thr, p->alias)) p->status = ORA_ENOMEM;
    return p;
}

ora_prep *ora_prepare(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w)
{
    return ora_prepare_model(n, m, row_ptr, col, w, 0);
}

int ora_prep_status(const ora_prep *p) { return p ? p->status : ORA_ENOMEM; }

void ora_prep_scalars(const ora_prep *p, double *Gamma, uint64_t *C)
{
    *Gamma = p->Gamma;
    *C = p->C;
}

/* Copies P[m], q[n], W[n], thr[n], alias[n] out of the preprocessing (any may be NULL). */
void ora_prep_copy(const ora_prep *p, double *P, double *q, uint64_t *W, uint64_t *thr, int32_t *alias)
{
    const size_t n = (size_t)p->n, m = (size_t)p->m;
    if (P && m) memcpy(P, p->P, sizeof(double) * m);
    if (q) memcpy(q, p->q, sizeof(double) * n);
    if (W) memcpy(W, p->W, sizeof(uint64_t) * n);
    if (thr && p->C) memcpy(thr, p->thr, sizeof(uint64_t) * n);
    if (alias && p->C) memcpy(alias, p->alias, sizeof(int32_t) * n);
}

/* Samples [j0, j1) with `nthreads` threads over contiguous id ranges; the result does not
 * depend on the thread count because sample j depends only on (graph, seed, j).
 * ris_mode = 1 draws plain RIS samples instead (singular ones included). */
ora_sketch *ora_sample(const ora_prep *p, uint64_t seed, uint64_t j0, uint64_t j1, int nthreads, int ris_mode)
{
    ora_sketch *sk = (ora_sketch *)calloc(1, sizeof(ora_sketch));
    if (!sk) return NULL;
    sk->j0 = j0;
    sk->j1 = j1;
    if (p->status < 0) { sk->status = p->status; return sk; }
    if (p->model == 1 && ris_mode) { sk->status = ORA_EINVAL; return sk; }
    sk->Gamma = p->Gamma;
    sk->C = p->C;
    uint64_t count = j1 > j0 ? j1 - j0 : 0;
    int64_t *sizes = NULL;
    sk->sample_ptr = (int64_t *)calloc((size_t)count + 1, sizeof(int64_t));
    sk->roots = (int32_t *)malloc(sizeof(int32_t) * (size_t)(count ? count : 1));
    sk->probed = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(count ? count : 1));
    sizes = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count ? count : 1));
    if (!sk->sample_ptr || !sk->roots || !sk->probed || !sizes) {
        sk->status = ORA_ENOMEM;
        goto done;
    }
    if (p->status == ORA_WDEGENERATE && !ris_mode) {
        /* No non-singular sample exists (Gamma = 0): an empty sketch. */
        sk->status = ORA_WDEGENERATE;
        sk->j1 = sk->j0;
        sk->nodes = (int32_t *)malloc(sizeof(int32_t));
        goto done;
    }
    {
        ora_ctx ctx = {p->n, p->row_ptr, p->col, p->w, p->P, p->q, p->thr, p->alias, p->C, seed, ris_mode, p->model};
        if (nthreads < 1) nthreads = 1;
        if ((uint64_t)nthreads > count && count > 0) nthreads = (int)count;
        ora_worker *wks = (ora_worker *)calloc((size_t)nthreads, sizeof(ora_worker));
        pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
        if (!wks || !tids) { free(wks); free(tids); sk->status = ORA_ENOMEM; goto done; }
        for (int t = 0; t < nthreads; ++t) {
            wks[t].g = &ctx;
            wks[t].j0 = j0 + count * (uint64_t)t / (uint64_t)nthreads;
            wks[t].j1 = j0 + count * (uint64_t)(t + 1) / (uint64_t)nthreads;
            wks[t].sizes = sizes + (wks[t].j0 - j0);
            wks[t].roots = sk->roots + (wks[t].j0 - j0);
            wks[t].probed = sk->probed + (wks[t].j0 - j0);
        }
        for (int t = 1; t < nthreads; ++t) pthread_create(&tids[t], NULL, ora_worker_run, &wks[t]);
        ora_worker_run(&wks[0]);
        for (int t = 1; t < nthreads; ++t) pthread_join(tids[t], NULL);
        int64_t total = 0;
        for (int t = 0; t < nthreads; ++t) {
            if (wks[t].status) sk->status = wks[t].status;
            total += wks[t].out.len;
        }
        if (!sk->status) {
            sk->nodes = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total ? total : 1));
            if (!sk->nodes) sk->status = ORA_ENOMEM;
        }
        if (!sk->status) {
            int64_t off = 0;
            for (int t = 0; t < nthreads; ++t) {
                if (wks[t].out.len)
                    memcpy(sk->nodes + off, wks[t].out.nodes, sizeof(int32_t) * (size_t)wks[t].out.len);
                off += wks[t].out.len;
            }
            for (uint64_t i = 0; i < count; ++i) {
                sk->sample_ptr[i + 1] = sk->sample_ptr[i] + sizes[i];
                sk->probed_total += sk->probed[i];
            }
            sk->entries = total;
        }
        for (int t = 0; t < nthreads; ++t) free(wks[t].out.nodes);
        free(wks);
        free(tids);
    }
done:
    free(sizes);
    return sk;
}

/* Preprocessing and samples [j0, j1) in one call. */
ora_sketch *ora_build(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                      const float *w, uint64_t seed, uint64_t j0, uint64_t j1, int nthreads,
                      int ris_mode)
{
    ora_prep *p = ora_prepare(n, m, row_ptr, col, w);
    if (!p) return NULL;
    ora_sketch *sk = ora_sample(p, seed, j0, j1, nthreads, ris_mode);
    ora_prep_free(p);
    return sk;
}

int ora_sketch_status(const ora_sketch *s) { return s ? s->status : ORA_ENOMEM; }

void ora_sketch_info(const ora_sketch *s, uint64_t *count, int64_t *entries, uint64_t *probed_total,
                     double *Gamma, uint64_t *C)
{
    *count = s->j1 - s->j0;
    *entries = s->entries;
    *probed_total = s->probed_total;
    *Gamma = s->Gamma;
    *C = s->C;
}

void ora_sketch_copy(const ora_sketch *s, int64_t *sample_ptr, int32_t *nodes, int32_t *roots, uint64_t *probed)
{
    uint64_t count = s->j1 - s->j0;
    memcpy(sample_ptr, s->sample_ptr, sizeof(int64_t) * (size_t)(count + 1));
    if (s->entries) memcpy(nodes, s->nodes, sizeof(int32_t) * (size_t)s->entries);
    if (count) {
        memcpy(roots, s->roots, sizeof(int32_t) * (size_t)count);
        memcpy(probed, s->probed, sizeof(uint64_t) * (size_t)count);
    }
}

/* ------------------------------------------------------------------------------------
 * Node -> samples incidence H(v) = { j : v in R_j }, the transpose of the sketch, each
 * list ascending in j (it is filled in sample order).  Used by the greedy's marginal
 * coverage Delta (Alg. 3, Eq. margin).
 * ---------------------------------------------------------------------------------- */
void ora_inverse(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes,
                 int64_t *node_ptr, int32_t *node_samples)
{
    memset(node_ptr, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < sample_ptr[T]; ++i) node_ptr[nodes[i] + 1]++;
    for (int32_t v = 0; v < n; ++v) node_ptr[v + 1] += node_ptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, node_ptr, sizeof(int64_t) * ((size_t)n + 1));
    for (uint64_t j = 0; j < T; ++j)
        for (int64_t i = sample_ptr[j]; i < sample_ptr[j + 1]; ++i)
            node_samples[fill[nodes[i]]++] = (int32_t)j;
    free(fill);
}

/* Compensated (Neumaier) sum of doubles, in the order given. */
static double neumaier(const double *x, int64_t k)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
        else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* Estimator of Eq. (eq21): I_hat(S) = Cov(S)/T * Gamma + sum_{v in S} (1 - gamma_v), with
 * S taken as a set (duplicates collapsed) and 1 - gamma_v read as q_v.  Cov is counted
 * straight from its definition in Table 1: the samples R_j that meet S.  For an empty
 * sketch (T = 0, Gamma = 0) the first term is 0. */
int ora_estimate(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes,
                 const double *q, double Gamma, int32_t Q, const int64_t *set_ptr,
                 const int32_t *set_nodes, uint64_t *cov_out, double *est_out)
{
    unsigned char *in_s = (unsigned char *)calloc((size_t)n, 1);
    if (!in_s) return ORA_ENOMEM;
    for (int32_t i = 0; i < Q; ++i) {
        int64_t a = set_ptr[i], b = set_ptr[i + 1];
        for (int64_t t = a; t < b; ++t)
            if (set_nodes[t] < 0 || set_nodes[t] >= n) { free(in_s); return ORA_EINVAL; }
        for (int64_t t = a; t < b; ++t) in_s[set_nodes[t]] = 1;
        uint64_t cov = 0;
        for (uint64_t j = 0; j < T; ++j) {
            for (int64_t p = sample_ptr[j]; p < sample_ptr[j + 1]; ++p)
                if (in_s[nodes[p]]) { ++cov; break; }
        }
        /* q over the distinct members of S, ascending by node id */
        int64_t k = 0;
        double *qs = (double *)malloc(sizeof(double) * (size_t)(b - a + 1));
        for (int32_t v = 0; v < n; ++v)
            if (in_s[v]) qs[k++] = q[v];
        double est = T > 0 ? ((double)cov * Gamma) / (double)T : 0.0;
        est_out[i] = est + neumaier(qs, k);
        cov_out[i] = cov;
        free(qs);
        for (int64_t t = a; t < b; ++t) in_s[set_nodes[t]] = 0;
    }
    free(in_s);
    return ORA_OK;
}

/* ------------------------------------------------------------------------------------
 * Alg. 3 (Greedy on the sketch).  Each of k rounds picks the node outside S_hat with the
 * largest gain Delta(v)/T * Gamma + q_v (Eq. margin), ties to the smallest id, then
 * marks the samples it newly covers and lowers Delta of every member of those samples.
 * Outputs: seeds in pick order, marginal coverage of each pick, total Cov, I_hat(S_hat).
 * ---------------------------------------------------------------------------------- */
int ora_greedy(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes,
               const double *q, double Gamma, int32_t k, int32_t *seeds, uint64_t *marg,
               uint64_t *cov_out, double *est_out)
{
    if (k < 1 || k > n) return ORA_EINVAL;
    int64_t E = sample_ptr[T];
    int64_t *node_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *node_samples = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
    int64_t *delta = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *covered = (unsigned char *)calloc((size_t)(T ? T : 1), 1);
    unsigned char *chosen = (unsigned char *)calloc((size_t)n, 1);
    double *qs = (double *)malloc(sizeof(double) * (size_t)k);
    if (!node_ptr || !node_samples || !delta || !covered || !chosen || !qs) {
        free(node_ptr); free(node_samples); free(delta); free(covered); free(chosen); free(qs);
        return ORA_ENOMEM;
    }
    ora_inverse(n, T, sample_ptr, nodes, node_ptr, node_samples);
    for (int32_t v = 0; v < n; ++v) delta[v] = node_ptr[v + 1] - node_ptr[v];
    uint64_t cov = 0;
    for (int32_t it = 0; it < k; ++it) {
        int32_t best = -1;
        double best_gain = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            if (chosen[v]) continue;
            double gain = (T > 0 ? ((double)delta[v] * Gamma) / (double)T : 0.0) + q[v];
            if (best < 0 || gain > best_gain) { best = v; best_gain = gain; }
        }
        seeds[it] = best;
        marg[it] = (uint64_t)delta[best];
        chosen[best] = 1;
        cov += (uint64_t)delta[best];
        for (int64_t p = node_ptr[best]; p < node_ptr[best + 1]; ++p) {
            int32_t j = node_samples[p];
            if (covered[j]) continue;
            covered[j] = 1;
            for (int64_t t = sample_ptr[j]; t < sample_ptr[j + 1]; ++t) delta[nodes[t]]--;
        }
    }
    int64_t kk = 0;
    for (int32_t v = 0; v < n; ++v)
        if (chosen[v]) qs[kk++] = q[v];
    *cov_out = cov;
    *est_out = (T > 0 ? ((double)cov * Gamma) / (double)T : 0.0) + neumaier(qs, kk);
    free(node_ptr); free(node_samples); free(delta); free(covered); free(chosen); free(qs);
    return ORA_OK;
}
