/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver that runs every routine of the CPU
 * oracle (skis_oracle.c, compiled into the same program) on small random graphs, so that the
 * oracle can be built and run under AddressSanitizer and UndefinedBehaviorSanitizer.  It
 * checks a few invariants on the way (alias mass, sample sizes, coverage bounds) and exits 0
 * when every one holds; any sanitizer report aborts the run.
 *
 * Build: gcc -O1 -g -std=gnu11 -fsanitize=address,undefined -fno-sanitize-recover=all
 *        -pthread sanitize_check.c skis_oracle.c -lm
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's entry points (skis_oracle.c) */
typedef struct ora_prep ora_prep_t;
typedef struct ora_sketch_s ora_sketch_t;
void ora_row_prefix(int32_t n, const int32_t *row_ptr, const float *w, double *P, double *q);
double ora_gamma_total(int32_t n, const double *q);
uint64_t ora_root_weights(int32_t n, const double *q, uint64_t *W);
int ora_alias_build(int32_t n, const uint64_t *W, uint64_t C, uint64_t *thr, int32_t *alias);
int ora_validate(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w);
void *ora_prepare(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w);
void *ora_prepare_model(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                        int model);
int ora_row_sums_lt(int32_t n, const int32_t *row_ptr, const float *w, double *S, double *q);
int ora_prep_status(const void *p);
void ora_prep_free(void *p);
void *ora_sample(const void *p, uint64_t seed, uint64_t j0, uint64_t j1, int nthreads, int ris_mode);
int ora_sketch_status(const void *s);
void ora_sketch_info(const void *s, uint64_t *count, int64_t *entries, uint64_t *probed_total, double *Gamma,
                     uint64_t *C);
void ora_sketch_copy(const void *s, int64_t *sample_ptr, int32_t *nodes, int32_t *roots, uint64_t *probed);
void ora_sketch_free(void *s);
void ora_inverse(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes, int64_t *node_ptr,
                 int32_t *node_samples);
int ora_estimate(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes, const double *q,
                 double Gamma, int32_t Q, const int64_t *set_ptr, const int32_t *set_nodes, uint64_t *cov_out,
                 double *est_out);
int ora_greedy(int32_t n, uint64_t T, const int64_t *sample_ptr, const int32_t *nodes, const double *q,
               double Gamma, int32_t k, int32_t *seeds, uint64_t *marg, uint64_t *cov_out, double *est_out);

static uint64_t lcg = 0x2545F4914F6CDD1Dull;
static uint32_t rnd(uint32_t bound)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(((lcg >> 33) * (uint64_t)bound) >> 31);
}

#define CHECK(c)                                                                                                 \
    do {                                                                                                         \
        if (!(c)) {                                                                                              \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);                                     \
            exit(1);                                                                                             \
        }                                                                                                        \
    } while (0)

/* A random graph in in-CSR form: n nodes, about m edges, rows by target, no self-loops. */
static void random_graph(int32_t n, int32_t m, int wc, int32_t **rp_out, int32_t **col_out, float **w_out, int64_t *m_out)
{
    int32_t *deg = calloc((size_t)n, sizeof(int32_t));
    int32_t *src = malloc(sizeof(int32_t) * (size_t)m), *dst = malloc(sizeof(int32_t) * (size_t)m);
    int32_t k = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t u = (int32_t)rnd((uint32_t)n), v = (int32_t)rnd((uint32_t)n);
        if (u == v) continue;
        src[k] = u;
        dst[k] = v;
        deg[v]++;
        ++k;
    }
    int32_t *rp = malloc(sizeof(int32_t) * ((size_t)n + 1));
    rp[0] = 0;
    for (int32_t v = 0; v < n; ++v) rp[v + 1] = rp[v] + deg[v];
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, rp, sizeof(int32_t) * (size_t)n);
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(k ? k : 1));
    float *w = malloc(sizeof(float) * (size_t)(k ? k : 1));
    static const float tri[3] = {0.1f, 0.01f, 0.001f};
    for (int32_t i = 0; i < k; ++i) {
        const int32_t p = fill[dst[i]]++;
        col[p] = src[i];
        w[p] = wc ? 1.0f / (float)deg[dst[i]] : tri[rnd(3)];
    }
    free(deg); free(src); free(dst); free(fill);
    *rp_out = rp; *col_out = col; *w_out = w; *m_out = k;
}

/* The linear threshold sampler (Sec. 6): WC weights (rows sum to 1, long walks that end on
 * cycles) and WC weights scaled by a per-node factor in (0, 1) (short walks). */
static void run_lt(int32_t n, int32_t m, int scaled)
{
    int32_t *rp, *col;
    float *w;
    int64_t mm;
    random_graph(n, m, 1, &rp, &col, &w, &mm);
    if (scaled)
        for (int32_t v = 0; v < n; ++v) {
            const float f = (float)(1 + rnd(1000)) / 1001.0f;
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) w[e] *= f;
        }
    double *S = malloc(sizeof(double) * (size_t)(mm ? mm : 1)), *q = malloc(sizeof(double) * (size_t)n);
    CHECK(ora_row_sums_lt(n, rp, w, S, q) == 0);
    void *prep = ora_prepare_model(n, mm, rp, col, w, 1);
    CHECK(prep && ora_prep_status(prep) >= 0);
    void *sk = ora_sample(prep, 11, 0, 4000, 3, 0);
    CHECK(sk && ora_sketch_status(sk) >= 0);
    uint64_t cnt, ptot, CC;
    int64_t ent;
    double GG;
    ora_sketch_info(sk, &cnt, &ent, &ptot, &GG, &CC);
    int64_t *sp = malloc(sizeof(int64_t) * (cnt + 1));
    int32_t *nodes = malloc(sizeof(int32_t) * (size_t)(ent ? ent : 1));
    int32_t *roots = malloc(sizeof(int32_t) * (cnt ? cnt : 1));
    uint64_t *probed = malloc(sizeof(uint64_t) * (cnt ? cnt : 1));
    ora_sketch_copy(sk, sp, nodes, roots, probed);
    for (uint64_t j = 0; j < cnt; ++j) {
        CHECK(sp[j + 1] - sp[j] >= 2);
        for (int64_t t = sp[j] + 1; t < sp[j + 1]; ++t) CHECK(nodes[t - 1] < nodes[t]);
    }
    void *bad = ora_sample(prep, 11, 0, 10, 1, 1); /* RIS mode is not defined for LT */
    CHECK(bad && ora_sketch_status(bad) < 0);
    ora_sketch_free(bad);
    ora_sketch_free(sk);
    ora_prep_free(prep);
    free(sp); free(nodes); free(roots); free(probed); free(S); free(q); free(rp); free(col); free(w);
}

static void run_graph(int32_t n, int32_t m, int wc, int ris)
{
    int32_t *rp, *col;
    float *w;
    int64_t mm;
    random_graph(n, m, wc, &rp, &col, &w, &mm);
    CHECK(ora_validate(n, mm, rp, col, w) == 0);
    double *P = malloc(sizeof(double) * (size_t)(mm ? mm : 1)), *q = malloc(sizeof(double) * (size_t)n);
    ora_row_prefix(n, rp, w, P, q);
    const double G = ora_gamma_total(n, q);
    uint64_t *W = malloc(sizeof(uint64_t) * (size_t)n), *thr = malloc(sizeof(uint64_t) * (size_t)n);
    int32_t *alias = malloc(sizeof(int32_t) * (size_t)n);
    const uint64_t C = ora_root_weights(n, q, W);
    if (C > 0) {
        CHECK(ora_alias_build(n, W, C, thr, alias) == 0);
        /* every node owns exactly n * W_v units of mass */
        unsigned __int128 *mass = calloc((size_t)n, sizeof(unsigned __int128));
        for (int32_t b = 0; b < n; ++b) {
            CHECK(thr[b] <= C && alias[b] >= 0 && alias[b] < n);
            mass[b] += thr[b];
            mass[alias[b]] += C - thr[b];
        }
        for (int32_t v = 0; v < n; ++v) CHECK(mass[v] == (unsigned __int128)n * W[v]);
        free(mass);
    }
    void *prep = ora_prepare(n, mm, rp, col, w);
    CHECK(prep && ora_prep_status(prep) >= 0);
    const uint64_t T = 3000;
    void *sk = ora_sample(prep, 7, 0, T, 3, ris);
    CHECK(sk && ora_sketch_status(sk) >= 0);
    uint64_t cnt, ptot, CC;
    int64_t ent;
    double GG;
    ora_sketch_info(sk, &cnt, &ent, &ptot, &GG, &CC);
    CHECK(GG == G && CC == C);
    int64_t *sp = malloc(sizeof(int64_t) * (cnt + 1));
    int32_t *nodes = malloc(sizeof(int32_t) * (size_t)(ent ? ent : 1));
    int32_t *roots = malloc(sizeof(int32_t) * (cnt ? cnt : 1));
    uint64_t *probed = malloc(sizeof(uint64_t) * (cnt ? cnt : 1));
    ora_sketch_copy(sk, sp, nodes, roots, probed);
    for (uint64_t j = 0; j < cnt; ++j) {
        CHECK(sp[j + 1] - sp[j] >= (ris ? 1 : 2));
        for (int64_t t = sp[j] + 1; t < sp[j + 1]; ++t) CHECK(nodes[t - 1] < nodes[t]);
    }
    /* a second range from the same preparation: ids [1000, 1500) equal the slice of the first */
    void *sk2 = ora_sample(prep, 7, 1000, 1500, 2, ris);
    int64_t *sp2 = malloc(sizeof(int64_t) * 501);
    uint64_t cnt2, ptot2, C2;
    int64_t ent2;
    double G2;
    ora_sketch_info(sk2, &cnt2, &ent2, &ptot2, &G2, &C2);
    int32_t *nodes2 = malloc(sizeof(int32_t) * (size_t)(ent2 ? ent2 : 1));
    int32_t *roots2 = malloc(sizeof(int32_t) * 500);
    uint64_t *probed2 = malloc(sizeof(uint64_t) * 500);
    ora_sketch_copy(sk2, sp2, nodes2, roots2, probed2);
    if (cnt == T) {
        CHECK(cnt2 == 500 && sp2[500] == sp[1500] - sp[1000]);
        CHECK(memcmp(nodes2, nodes + sp[1000], sizeof(int32_t) * (size_t)ent2) == 0);
    }
    /* transpose, estimates, greedy */
    int64_t *np = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *ns = malloc(sizeof(int32_t) * (size_t)(ent ? ent : 1));
    ora_inverse(n, cnt, sp, nodes, np, ns);
    CHECK(np[n] == ent);
    int64_t set_ptr[4] = {0, 3, 3, 8};
    int32_t set_nodes[8] = {0, 1, 2, 3, 3, 4, 5, 6};
    for (int i = 0; i < 8; ++i) set_nodes[i] %= n;
    uint64_t cov[3];
    double est[3];
    CHECK(ora_estimate(n, cnt, sp, nodes, q, ris ? (double)n : G, 3, set_ptr, set_nodes, cov, est) == 0);
    for (int i = 0; i < 3; ++i) CHECK(cov[i] <= cnt && est[i] >= 0.0);
    int32_t seeds[5];
    uint64_t marg[5], gc;
    double ge;
    if (n >= 5) {
        CHECK(ora_greedy(n, cnt, sp, nodes, q, ris ? (double)n : G, 5, seeds, marg, &gc, &ge) == 0);
        uint64_t sum = 0;
        for (int i = 0; i < 5; ++i) sum += marg[i];
        CHECK(sum == gc && gc <= cnt);
    }
    ora_sketch_free(sk);
    ora_sketch_free(sk2);
    ora_prep_free(prep);
    free(sp); free(nodes); free(roots); free(probed); free(sp2); free(nodes2); free(roots2); free(probed2);
    free(np); free(ns); free(P); free(q); free(W); free(thr); free(alias); free(rp); free(col); free(w);
}

int main(void)
{
    run_graph(200, 1500, 1, 0);
    run_graph(200, 1500, 0, 0);
    run_graph(1000, 3000, 1, 0);
    run_graph(300, 2000, 0, 1);
    run_graph(5, 8, 1, 0);
    run_graph(3, 2, 0, 1);
    run_lt(300, 2000, 0);
    run_lt(300, 2000, 1);
    run_lt(4, 5, 0);
    printf("sanitized oracle run ok\n");
    return 0;
}
