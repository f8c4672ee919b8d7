/*
 * Exact 0/1 knapsack references -- TEST INFRASTRUCTURE ONLY.
 *
 * These do not implement QIEO; they pin it.  Eq. (1) of the paper defines
 * the fitness that QIEO maximises; its maximum over all strings is the
 * knapsack optimum, which these routines compute by textbook methods that
 * share nothing with the evolutionary loop:
 *   - knap_bruteforce: enumerate all 2^n strings (n <= 24), scoring each
 *     with eq. (1) written out independently here;
 *   - knap_dp: the classical O(n*C) dynamic program over capacities;
 *   - knap_lp_bound: Dantzig's fractional (LP-relaxation) upper bound.
 */
#include <stdint.h>
#include <stdlib.h>

/* Eq. (1) for one string given as a bitmask (bit i = item i). */
static int64_t fitness_mask(int n, const int32_t *v, const int32_t *w, int64_t cap,
                            int64_t lambda, uint64_t mask)
{
    int64_t P = 0, W = 0;
    for (int i = 0; i < n; ++i) {
        if ((mask >> i) & 1u) { P += v[i]; W += w[i]; }
    }
    if (W <= cap) return P;
    return -lambda * (W - cap);
}

/* Maximum of eq. (1) over all 2^n strings; writes the lowest maximising mask. */
int64_t knap_bruteforce(int n, const int32_t *v, const int32_t *w, int64_t cap,
                        int64_t lambda, uint64_t *argmax)
{
    if (n < 0 || n > 24) return INT64_MIN;
    uint64_t best_m = 0;
    int64_t best = fitness_mask(n, v, w, cap, lambda, 0);
    for (uint64_t m = 1; m < ((uint64_t)1 << n); ++m) {
        int64_t f = fitness_mask(n, v, w, cap, lambda, m);
        if (f > best) { best = f; best_m = m; }
    }
    if (argmax) *argmax = best_m;
    return best;
}

/* Fitness of every one of the 2^n strings (out has 2^n entries). */
int knap_all_fitness(int n, const int32_t *v, const int32_t *w, int64_t cap,
                     int64_t lambda, int64_t *out)
{
    if (n < 0 || n > 24) return -1;
    for (uint64_t m = 0; m < ((uint64_t)1 << n); ++m)
        out[m] = fitness_mask(n, v, w, cap, lambda, m);
    return 0;
}

/* Classical dynamic program: best[c] = max profit with total weight <= c. */
int64_t knap_dp(int n, const int32_t *v, const int32_t *w, int64_t cap)
{
    if (cap < 0) return -1;
    int64_t *best = (int64_t *)calloc((size_t)cap + 1, sizeof(int64_t));
    if (!best) return -2;
    for (int i = 0; i < n; ++i) {
        int64_t wi = w[i];
        if (wi > cap) continue;
        for (int64_t c = cap; c >= wi; --c) {
            int64_t cand = best[c - wi] + v[i];
            if (cand > best[c]) best[c] = cand;
        }
    }
    int64_t r = best[cap];
    free(best);
    return r;
}

static const int32_t *g_v, *g_w;
static int cmp_ratio(const void *a, const void *b)
{
    int ia = *(const int *)a, ib = *(const int *)b;
    /* descending v/w; cross-multiplied in 64-bit to stay exact */
    int64_t l = (int64_t)g_v[ia] * g_w[ib];
    int64_t r = (int64_t)g_v[ib] * g_w[ia];
    if (l > r) return -1;
    if (l < r) return 1;
    return ia - ib;
}

/* Dantzig's bound: fill by decreasing value density, last item fractional. */
double knap_lp_bound(int n, const int32_t *v, const int32_t *w, int64_t cap)
{
    int *idx = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!idx) return -1.0;
    for (int i = 0; i < n; ++i) idx[i] = i;
    g_v = v; g_w = w;
    qsort(idx, (size_t)n, sizeof(int), cmp_ratio);
    double room = (double)cap, val = 0.0;
    for (int k = 0; k < n; ++k) {
        int i = idx[k];
        if (w[i] == 0) { val += v[i]; continue; }
        if (w[i] <= room) { room -= w[i]; val += v[i]; }
        else { val += v[i] * (room / w[i]); break; }
    }
    free(idx);
    return val;
}
