/*
 * Drives every entry point of the CPU oracle (oracle/qieo_oracle.c,
 * oracle/knapsack_exact.c) on small instances, built by
 * tests/test_host_sanitized.py with gcc under the address and
 * undefined-behaviour sanitizers (with the oracle's own flags: no FP
 * contraction, no fast-math).  Besides memory and UB errors, which the
 * sanitizers report, it checks a few properties that tie the entry points
 * together: the row-local step reproduces the population step, threads do
 * not change the state, the best record is monotone and below the exact
 * optimum, and the norm stays within 1e-5.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle oracle;
oracle *oracle_new(int32_t ng, int32_t np, const int32_t *v, const int32_t *w, int64_t cap,
                   uint64_t seed, int64_t lambda);
oracle *oracle_new_f64(int32_t ng, int32_t np, const int32_t *v, const int32_t *w, int64_t cap,
                       uint64_t seed, int64_t lambda);
void oracle_free(oracle *s);
void oracle_set_threads(oracle *s, int threads);
void oracle_generation(oracle *s);
void oracle_run(oracle *s, int64_t n);
int oracle_converged(const oracle *s, int window);
int64_t oracle_run_until_converged(oracle *s, int64_t n, int window);
void oracle_get_amplitudes(const oracle *s, float *alpha, float *beta);
void oracle_get_amplitudes_f64(const oracle *s, double *alpha, double *beta);
void oracle_set_amplitudes(oracle *s, const float *alpha, const float *beta);
void oracle_set_amplitudes_f64(oracle *s, const double *alpha, const double *beta);
void oracle_get_alleles(const oracle *s, uint8_t *x);
void oracle_set_alleles(oracle *s, const uint8_t *x);
void oracle_get_fitness(const oracle *s, int64_t *fit, int64_t *P, int64_t *W);
void oracle_set_fitness(oracle *s, const int64_t *fit);
int64_t oracle_generation_index(const oracle *s);
int64_t oracle_elite(const oracle *s);
void oracle_get_best(const oracle *s, int64_t out[6], uint8_t *bits);
void oracle_row_generation(uint64_t seed, int64_t t, int64_t c, int64_t ng, const int32_t *v,
                           const int32_t *w, int64_t cap, float *alpha, float *beta,
                           const uint8_t *x_prev, const uint8_t *elite_prev, int below_elite,
                           uint8_t *x_out, int64_t out[3]);
void oracle_row_generation_f64(uint64_t seed, int64_t t, int64_t c, int64_t ng, const int32_t *v,
                               const int32_t *w, int64_t cap, double *alpha, double *beta,
                               const uint8_t *x_prev, const uint8_t *elite_prev, int below_elite,
                               uint8_t *x_out, int64_t out[3]);
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float oracle_uniform(uint64_t seed, int64_t t, int64_t c, int64_t i);
int oracle_cip_gene(float *alpha, float *beta, int tgt);
int oracle_cip_gene_f64(double *alpha, double *beta, int tgt);
int64_t knap_bruteforce(int n, const int32_t *v, const int32_t *w, int64_t cap, int64_t lambda,
                        uint64_t *mask);
int knap_all_fitness(int n, const int32_t *v, const int32_t *w, int64_t cap, int64_t lambda,
                     int64_t *out);
int64_t knap_dp(int n, const int32_t *v, const int32_t *w, int64_t cap);
double knap_lp_bound(int n, const int32_t *v, const int32_t *w, int64_t cap);

#define CHECK(cond, msg)                                                       \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "FAIL %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, msg); \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

static uint64_t lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return *s >> 33;
}

/* Items with weights in [1, wmax], value = weight + off, capacity half the
 * weight sum (the correlated generator of the workloads, drawn here with a
 * plain LCG: only the shapes matter to these checks). */
static int64_t items(int n, int32_t *v, int32_t *w, uint64_t seed, int wmax, int off)
{
    int64_t sum = 0;
    for (int i = 0; i < n; ++i) {
        w[i] = 1 + (int32_t)(lcg(&seed) % (uint64_t)wmax);
        v[i] = w[i] + off;
        sum += w[i];
    }
    return sum / 2;
}

static void run_population(int ng, int np, int gens, int f64, int threads)
{
    int32_t *v = malloc(sizeof(int32_t) * ng), *w = malloc(sizeof(int32_t) * ng);
    const int64_t cap = items(ng, v, w, 99 + ng, 10, 5);
    oracle *a = f64 ? oracle_new_f64(ng, np, v, w, cap, 5, 1) : oracle_new(ng, np, v, w, cap, 5, 1);
    oracle *b = f64 ? oracle_new_f64(ng, np, v, w, cap, 5, 1) : oracle_new(ng, np, v, w, cap, 5, 1);
    CHECK(a && b, "oracle_new");
    oracle_set_threads(b, threads);
    const size_t n = (size_t)ng * np;
    double *ad = malloc(sizeof(double) * n), *bd = malloc(sizeof(double) * n);
    float *af = malloc(sizeof(float) * n), *bf = malloc(sizeof(float) * n);
    double *ad2 = malloc(sizeof(double) * n), *bd2 = malloc(sizeof(double) * n);
    float *af2 = malloc(sizeof(float) * n), *bf2 = malloc(sizeof(float) * n);
    uint8_t *x = malloc(n), *x2 = malloc(n), *bits = malloc((size_t)ng);
    int64_t *fit = malloc(sizeof(int64_t) * np), *P = malloc(sizeof(int64_t) * np);
    int64_t *W = malloc(sizeof(int64_t) * np), *fit2 = malloc(sizeof(int64_t) * np);
    int64_t best_prev = INT64_MIN, rec[6];
    /* row-local replay of every chromosome: amplitudes, previous alleles */
    float *ra = malloc(sizeof(float) * n), *rb = malloc(sizeof(float) * n);
    double *rad = malloc(sizeof(double) * n), *rbd = malloc(sizeof(double) * n);
    uint8_t *rx = calloc(n, 1), *rx2 = calloc(n, 1), *elite_x = calloc((size_t)ng, 1);
    int64_t *rfit = calloc((size_t)np, sizeof(int64_t)), fe = 0;
    if (f64) oracle_get_amplitudes_f64(a, rad, rbd);
    else oracle_get_amplitudes(a, ra, rb);
    for (int g = 0; g < gens; ++g) {
        oracle_generation(a);
        oracle_run(b, 1);
        const int64_t t = oracle_generation_index(a) - 1;
        for (int c = 0; c < np; ++c) {
            int64_t out[3];
            const int below = t > 0 && rfit[c] < fe;
            if (f64)
                oracle_row_generation_f64(5, t, c, ng, v, w, cap, rad + (size_t)c * ng,
                                          rbd + (size_t)c * ng, rx + (size_t)c * ng, elite_x,
                                          below, rx2 + (size_t)c * ng, out);
            else
                oracle_row_generation(5, t, c, ng, v, w, cap, ra + (size_t)c * ng,
                                      rb + (size_t)c * ng, rx + (size_t)c * ng, elite_x, below,
                                      rx2 + (size_t)c * ng, out);
            rfit[c] = out[0];
        }
        memcpy(rx, rx2, n);
        oracle_get_fitness(a, fit, P, W);
        oracle_get_fitness(b, fit2, NULL, NULL);
        oracle_get_alleles(a, x);
        oracle_get_alleles(b, x2);
        CHECK(memcmp(fit, fit2, sizeof(int64_t) * np) == 0, "threads change fitness");
        CHECK(memcmp(x, x2, n) == 0, "threads change alleles");
        CHECK(memcmp(fit, rfit, sizeof(int64_t) * np) == 0, "row step differs in fitness");
        CHECK(memcmp(x, rx, n) == 0, "row step differs in alleles");
        const int64_t e = oracle_elite(a);
        CHECK(e >= 0 && e < np, "elite index");
        for (int c = 0; c < np; ++c)
            CHECK(fit[c] < fit[e] || (fit[c] == fit[e] && c >= e), "elite is the argmax");
        fe = fit[e];
        memcpy(elite_x, x + (size_t)e * ng, (size_t)ng);
        oracle_get_best(a, rec, bits);
        CHECK(rec[0] == 1 && rec[1] >= best_prev, "best record monotone");
        best_prev = rec[1];
        if (f64) {
            oracle_get_amplitudes_f64(a, ad, bd);
            oracle_get_amplitudes_f64(b, ad2, bd2);
            CHECK(memcmp(ad, ad2, sizeof(double) * n) == 0 && memcmp(bd, bd2, sizeof(double) * n) == 0,
                  "threads change amplitudes");
            for (size_t k = 0; k < n; ++k)
                CHECK(fabs(ad[k] * ad[k] + bd[k] * bd[k] - 1.0) <= 1e-5, "norm");
        } else {
            oracle_get_amplitudes(a, af, bf);
            oracle_get_amplitudes(b, af2, bf2);
            CHECK(memcmp(af, af2, sizeof(float) * n) == 0 && memcmp(bf, bf2, sizeof(float) * n) == 0,
                  "threads change amplitudes");
            for (size_t k = 0; k < n; ++k)
                CHECK(fabs((double)af[k] * af[k] + (double)bf[k] * bf[k] - 1.0) <= 1e-5, "norm");
        }
    }
    if (ng <= 24) CHECK(rec[1] <= knap_dp(ng, v, w, cap), "best above the optimum");
    /* setters round-trip */
    if (f64) {
        oracle_set_amplitudes_f64(b, ad, bd);
    } else {
        oracle_set_amplitudes(b, af, bf);
    }
    oracle_set_alleles(b, x);
    oracle_set_fitness(b, fit);
    /* convergence on a copy: stops at most at the cap and stays stopped */
    const int64_t ran = oracle_run_until_converged(b, 50, 3);
    CHECK(ran >= 0 && ran <= 50, "run_until_converged cap");
    if (oracle_converged(b, 3)) CHECK(oracle_run_until_converged(b, 10, 3) == 0, "restart");
    oracle_free(a);
    oracle_free(b);
    free(v); free(w); free(ad); free(bd); free(af); free(bf); free(ad2); free(bd2);
    free(af2); free(bf2); free(x); free(x2); free(bits); free(fit); free(P); free(W);
    free(fit2); free(ra); free(rb); free(rad); free(rbd); free(rx); free(rx2); free(elite_x);
    free(rfit);
}

static void knapsack_refs(void)
{
    for (int n = 1; n <= 14; ++n) {
        int32_t v[14], w[14];
        const int64_t cap = items(n, v, w, 1234 + n, 10, 5);
        uint64_t mask = 0;
        const int64_t bf = knap_bruteforce(n, v, w, cap, 1, &mask);
        CHECK(bf == knap_dp(n, v, w, cap), "brute force vs DP");
        CHECK(knap_lp_bound(n, v, w, cap) >= (double)bf, "LP bound");
        int64_t *all = malloc(sizeof(int64_t) << n);
        CHECK(knap_all_fitness(n, v, w, cap, 1, all) == 0, "all fitness");
        int64_t m = INT64_MIN;
        for (int64_t k = 0; k < ((int64_t)1 << n); ++k) m = all[k] > m ? all[k] : m;
        CHECK(m == bf, "enumeration max");
        free(all);
    }
}

static void single_steps(void)
{
    const uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    CHECK(out[0] == 0x6627e8d5u && out[3] == 0x9b00dbd8u, "Philox known answer");
    for (int64_t i = 0; i < 64; ++i) {
        const float u = oracle_uniform(3, 1, 2, i);
        CHECK(u >= 0.0f && u < 1.0f, "uniform range");
    }
    float a = 0x1.6a09e6p-1f, b = 0x1.6a09e6p-1f;
    double ad = 0x1.6a09e667f3bcdp-1, bd = ad;
    for (int k = 0; k < 100; ++k) {
        CHECK(oracle_cip_gene(&a, &b, k & 1) == 1, "rotation");
        CHECK(oracle_cip_gene_f64(&ad, &bd, k & 1) == 1, "rotation f64");
    }
    a = 0.0f; b = 1.0f;
    CHECK(oracle_cip_gene(&a, &b, 1) == 0, "pole skip");
    ad = 1.0; bd = 0.0;
    CHECK(oracle_cip_gene_f64(&ad, &bd, 0) == 0, "pole skip f64");
}

int main(void)
{
    single_steps();
    knapsack_refs();
    const int shapes[][3] = {{1, 1, 12}, {3, 5, 20}, {20, 16, 40}, {100, 16, 60}, {257, 7, 30},
                             {1000, 3, 15}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (int f64 = 0; f64 <= 1; ++f64)
            run_population(shapes[s][0], shapes[s][1], shapes[s][2], f64, 3);
    printf("oracle checks passed\n");
    return 0;
}
