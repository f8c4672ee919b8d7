/*
 * QIEO oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded (optionally row-threaded) CPU implementation
 * of one generation of quantum-inspired evolutionary optimization on the
 * 0/1 knapsack problem, written from the paper "Evaluation of portability and
 * performance of an OpenMP5 offloaded Quantum-Inspired Evolutionary
 * Optimization Across the GPU Ecosystem" (Srikanth et al.):
 *   - the qubit gene and its norm constraint (Sec. I, Introduction),
 *   - the knapsack fitness, eq. (1) (Sec. III-A, Formulation),
 *   - the four steps QIP -> Evaluation -> DetermineElite -> CIP and their
 *     order (Sec. III-B, Methodology, and Fig. 1).
 * Where the paper is silent, the readings below are the ones the GPU library
 * implements as well (they are its specification, not borrowed code):
 *   R1  allele 1 is observed iff u < beta^2, u a 24-bit uniform in [0,1).
 *   R2  QIP only reads the amplitudes; CIP (rotation + renormalisation) is
 *       their only writer.
 *   R3  CIP rotates gene i of chromosome c only when f(c) < f(elite) and
 *       x[c][i] != b[i] (b = elite string), by |dtheta| = 0.01*pi, with the
 *       sign chosen from the quadrant of (alpha, beta) so that beta^2 moves
 *       toward b[i]; a zero product takes the fixed rule in cip_gene().
 *   R4  the rotation is followed by one Newton step toward unit norm,
 *       g = 1.5 - 0.5*n, using only +, -, * (bit-reproducible everywhere).
 *   R5  the elite is the generation best; ties go to the lowest index.
 *   R6  FP32 amplitudes initialised to fl32(1/sqrt 2); exact integer fitness.
 *   R7  uniform draws come from Philox4x32-10 (Salmon et al., SC'11) with
 *       counter {i/4, c, t, 0} and key {seed_lo, seed_hi}; gene i uses word
 *       i mod 4 of its call.
 *
 *   R8  (binary64 variant, the paper's precision, Sec. V) the same steps on
 *       binary64 amplitudes with binary64 roundings of the same constants;
 *       the uniform draw stays the 24-bit value of R1.
 *
 * Every floating-point operation below is one IEEE-754 operation of the
 * amplitude precision, rounded to nearest (build with -ffp-contract=off, no
 * fast-math, SSE).
 *
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this code.  The GPU library shares nothing with it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror,       */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds   */
/* of two 32x32->64 multiplies with a Weyl-sequence key schedule.           */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The four 32-bit draws of genes 4k..4k+3 of chromosome c at generation t
 * (reading R7). */
static void draws4(uint64_t seed, int64_t t, int64_t c, int64_t k, uint32_t r[4])
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)c, (uint32_t)t, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, r);
}

/* 24-bit uniform in [0, 1 - 2^-24], exact in binary32 (reading R1). */
static float uniform24(uint32_t r)
{
    return (float)(r >> 8) * 0x1p-24f;
}

float oracle_uniform(uint64_t seed, int64_t t, int64_t c, int64_t i)
{
    uint32_t r[4];
    draws4(seed, t, c, i / 4, r);
    return uniform24(r[i % 4]);
}

/* ------------------------------------------------------------------------ */
/* Rotation gate constants (reading R3): binary32 roundings of cos(0.01 pi), */
/* sin(0.01 pi) and 1/sqrt(2), written as exact hex literals.               */
/* ------------------------------------------------------------------------ */
#define ROT_C  0x1.ffbf52p-1f
#define ROT_S  0x1.015122p-5f
#define AMP0   0x1.6a09e6p-1f

/* binary64 roundings (correctly rounded) of the same three constants */
#define ROT_C64 0x1.ffbf52e9d1086p-1
#define ROT_S64 0x1.015122df75860p-5
#define AMP0_64 0x1.6a09e667f3bcdp-1

/* CIP on one gene (readings R3, R4).  tgt is the elite's allele b[i].
 * Returns 1 if the gene was rotated, 0 if the zero-product rule skipped it. */
int oracle_cip_gene(float *alpha, float *beta, int tgt)
{
    float a = *alpha, b = *beta;
    float p = a * b;
    float sd;
    if (p > 0.0f) {
        /* d(beta^2)/dtheta = 2 alpha beta > 0: positive angle raises beta^2 */
        sd = tgt ? ROT_S : -ROT_S;
    } else if (p < 0.0f) {
        sd = tgt ? -ROT_S : ROT_S;
    } else {
        /* on an axis: nothing to do if already at the target pole */
        if ((tgt && a == 0.0f) || (!tgt && b == 0.0f))
            return 0;
        sd = ROT_S;
    }
    float a1 = ROT_C * a - sd * b;
    float b1 = sd * a + ROT_C * b;
    float n = a1 * a1 + b1 * b1;
    float g = 1.5f - 0.5f * n;
    *alpha = a1 * g;
    *beta = b1 * g;
    return 1;
}

/* The same gate in binary64 (reading R8). */
int oracle_cip_gene_f64(double *alpha, double *beta, int tgt)
{
    double a = *alpha, b = *beta;
    double p = a * b;
    double sd;
    if (p > 0.0) {
        sd = tgt ? ROT_S64 : -ROT_S64;
    } else if (p < 0.0) {
        sd = tgt ? -ROT_S64 : ROT_S64;
    } else {
        if ((tgt && a == 0.0) || (!tgt && b == 0.0))
            return 0;
        sd = ROT_S64;
    }
    double a1 = ROT_C64 * a - sd * b;
    double b1 = sd * a + ROT_C64 * b;
    double n = a1 * a1 + b1 * b1;
    double g = 1.5 - 0.5 * n;
    *alpha = a1 * g;
    *beta = b1 * g;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* State.                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct oracle {
    int32_t ng, np;
    int64_t cap;        /* knapsack capacity W of eq. (1) */
    int64_t lambda;     /* penalty factor of eq. (1), > 0 */
    uint64_t seed;
    int32_t *v, *w;     /* item values and weights, length ng */
    float *alpha, *beta;/* np x ng, chromosome-major */
    uint8_t *x;         /* observed alleles of the current generation */
    int64_t *P, *W, *fit;
    int64_t t;          /* index of the next generation to run */
    int64_t elite;      /* elite of the last completed generation, -1 none */
    int has_best;
    int64_t best_f, best_P, best_W, best_gen, best_chrom;
    uint8_t *best_x;
    int threads;
    int64_t *elite_f;   /* elite fitness of every completed generation */
    int64_t elite_cap;
    int f64;            /* binary64 amplitudes (reading R8) */
    double *alpha_d, *beta_d;
} oracle;

void oracle_free(oracle *s)
{
    if (!s) return;
    free(s->v); free(s->w); free(s->alpha); free(s->beta); free(s->x);
    free(s->P); free(s->W); free(s->fit); free(s->best_x); free(s->elite_f);
    free(s->alpha_d); free(s->beta_d);
    free(s);
}

/* Creates the initial population (every amplitude fl32(1/sqrt 2), reading
 * R6).  Returns NULL on bad sizes or allocation failure. */
oracle *oracle_new(int32_t ng, int32_t np, const int32_t *v, const int32_t *w,
                   int64_t cap, uint64_t seed, int64_t lambda)
{
    if (ng < 1 || np < 1 || lambda < 1) return NULL;
    oracle *s = (oracle *)calloc(1, sizeof(oracle));
    if (!s) return NULL;
    size_t n = (size_t)ng * (size_t)np;
    s->ng = ng; s->np = np; s->cap = cap; s->seed = seed; s->lambda = lambda;
    s->v = (int32_t *)malloc(sizeof(int32_t) * ng);
    s->w = (int32_t *)malloc(sizeof(int32_t) * ng);
    s->alpha = (float *)malloc(sizeof(float) * n);
    s->beta = (float *)malloc(sizeof(float) * n);
    s->x = (uint8_t *)calloc(n, 1);
    s->P = (int64_t *)calloc(np, sizeof(int64_t));
    s->W = (int64_t *)calloc(np, sizeof(int64_t));
    s->fit = (int64_t *)calloc(np, sizeof(int64_t));
    s->best_x = (uint8_t *)calloc(ng, 1);
    if (!s->v || !s->w || !s->alpha || !s->beta || !s->x || !s->P || !s->W ||
        !s->fit || !s->best_x) {
        oracle_free(s);
        return NULL;
    }
    memcpy(s->v, v, sizeof(int32_t) * ng);
    memcpy(s->w, w, sizeof(int32_t) * ng);
    for (size_t k = 0; k < n; ++k) { s->alpha[k] = AMP0; s->beta[k] = AMP0; }
    s->t = 0;
    s->elite = -1;
    s->has_best = 0;
    s->threads = 1;
    return s;
}

/* The binary64 variant: same problem, amplitudes fl64(1/sqrt 2). */
oracle *oracle_new_f64(int32_t ng, int32_t np, const int32_t *v, const int32_t *w,
                       int64_t cap, uint64_t seed, int64_t lambda)
{
    oracle *s = oracle_new(ng, np, v, w, cap, seed, lambda);
    if (!s) return NULL;
    size_t n = (size_t)ng * (size_t)np;
    s->alpha_d = (double *)malloc(sizeof(double) * n);
    s->beta_d = (double *)malloc(sizeof(double) * n);
    if (!s->alpha_d || !s->beta_d) {
        oracle_free(s);
        return NULL;
    }
    free(s->alpha); free(s->beta);
    s->alpha = NULL; s->beta = NULL;
    for (size_t k = 0; k < n; ++k) { s->alpha_d[k] = AMP0_64; s->beta_d[k] = AMP0_64; }
    s->f64 = 1;
    return s;
}

void oracle_set_threads(oracle *s, int threads) { s->threads = threads < 1 ? 1 : threads; }

/* QIP (Sec. III-B): observe every qubit of every chromosome (reading R1, R2). */
void oracle_qip(oracle *s)
{
    const int64_t ng = s->ng;
    const int64_t nk = (ng + 3) / 4;
#pragma omp parallel for num_threads(s->threads) schedule(static)
    for (int64_t c = 0; c < s->np; ++c) {
        for (int64_t k = 0; k < nk; ++k) {
            uint32_t r[4];
            draws4(s->seed, s->t, c, k, r);
            for (int j = 0; j < 4; ++j) {
                int64_t i = 4 * k + j;
                if (i >= ng) break;
                if (s->f64) {
                    double b = s->beta_d[c * ng + i];
                    double b2 = b * b;
                    double u = (double)(r[j] >> 8) * 0x1p-24;
                    s->x[c * ng + i] = (u < b2) ? 1 : 0;
                } else {
                    float b = s->beta[c * ng + i];
                    float b2 = b * b;
                    s->x[c * ng + i] = (uniform24(r[j]) < b2) ? 1 : 0;
                }
            }
        }
    }
}

/* Evaluation, eq. (1): profit and weight sums, then the capacity test; an
 * infeasible chromosome scores -lambda times its excess weight. */
void oracle_fe(oracle *s)
{
    const int64_t ng = s->ng;
#pragma omp parallel for num_threads(s->threads) schedule(static)
    for (int64_t c = 0; c < s->np; ++c) {
        int64_t P = 0, W = 0;
        for (int64_t i = 0; i < ng; ++i) {
            P += (int64_t)s->v[i] * s->x[c * ng + i];
            W += (int64_t)s->w[i] * s->x[c * ng + i];
        }
        s->P[c] = P;
        s->W[c] = W;
        s->fit[c] = (W <= s->cap) ? P : -s->lambda * (W - s->cap);
    }
}

/* DetermineElite (Sec. III-B): the generation-best chromosome, lowest index
 * on ties (reading R5); the best-so-far record changes only on a strictly
 * larger fitness. */
void oracle_de(oracle *s)
{
    int64_t e = 0;
    for (int64_t c = 1; c < s->np; ++c)
        if (s->fit[c] > s->fit[e]) e = c;
    s->elite = e;
    if (s->t >= s->elite_cap) {
        int64_t cap = s->elite_cap ? 2 * s->elite_cap : 1024;
        while (cap <= s->t) cap *= 2;
        int64_t *p = (int64_t *)realloc(s->elite_f, sizeof(int64_t) * (size_t)cap);
        if (p) { s->elite_f = p; s->elite_cap = cap; }
    }
    if (s->t < s->elite_cap) s->elite_f[s->t] = s->fit[e];
    if (!s->has_best || s->fit[e] > s->best_f) {
        s->has_best = 1;
        s->best_f = s->fit[e];
        s->best_P = s->P[e];
        s->best_W = s->W[e];
        s->best_gen = s->t;
        s->best_chrom = e;
        memcpy(s->best_x, s->x + e * (int64_t)s->ng, (size_t)s->ng);
    }
}

/* CIP (Sec. III-B): rotate every qubit of every chromosome that scores below
 * the elite toward the elite's allele where the two differ (reading R3). */
void oracle_cip(oracle *s)
{
    const int64_t ng = s->ng;
    const int64_t e = s->elite;
    const int64_t fe = s->fit[e];
    const uint8_t *b = s->x + e * ng;
#pragma omp parallel for num_threads(s->threads) schedule(static)
    for (int64_t c = 0; c < s->np; ++c) {
        if (!(s->fit[c] < fe)) continue;
        for (int64_t i = 0; i < ng; ++i) {
            if (s->x[c * ng + i] == b[i]) continue;
            if (s->f64)
                oracle_cip_gene_f64(&s->alpha_d[c * ng + i], &s->beta_d[c * ng + i], b[i]);
            else
                oracle_cip_gene(&s->alpha[c * ng + i], &s->beta[c * ng + i], b[i]);
        }
    }
}

/* One generation, in the order of Fig. 1. */
void oracle_generation(oracle *s)
{
    oracle_qip(s);
    oracle_fe(s);
    oracle_de(s);
    oracle_cip(s);
    s->t += 1;
}

void oracle_run(oracle *s, int64_t n)
{
    for (int64_t g = 0; g < n; ++g) oracle_generation(s);
}

/* One chromosome's part of generation t (binary32, lambda = 1).  Of the four
 * steps of Fig. 1 only DetermineElite looks across chromosomes; given the
 * elite of generation t-1 (its alleles, and whether chromosome c scored below
 * it), chromosome c's generation t is: CIP of t-1 toward the elite (readings
 * R3, R4), then QIP of t (R1, R7) and Evaluation, eq. (1).  alpha and beta
 * (ng each) hold c's amplitudes as generation t-1 observed them and receive
 * the rotated ones; x_prev and elite_prev are c's and the elite's alleles of
 * t-1 (not read when below_elite is 0, as at t = 0); x_out receives the
 * alleles of t; out = {fitness, profit, weight}.  Chromosome-local, so it
 * serves populations too large for the whole-population oracle. */
void oracle_row_generation(uint64_t seed, int64_t t, int64_t c, int64_t ng,
                           const int32_t *v, const int32_t *w, int64_t cap,
                           float *alpha, float *beta, const uint8_t *x_prev,
                           const uint8_t *elite_prev, int below_elite,
                           uint8_t *x_out, int64_t out[3])
{
    if (below_elite)
        for (int64_t i = 0; i < ng; ++i)
            if (x_prev[i] != elite_prev[i])
                oracle_cip_gene(&alpha[i], &beta[i], elite_prev[i]);
    int64_t P = 0, W = 0;
    for (int64_t k = 0; 4 * k < ng; ++k) {
        uint32_t r[4];
        draws4(seed, t, c, k, r);
        for (int j = 0; j < 4 && 4 * k + j < ng; ++j) {
            const int64_t i = 4 * k + j;
            const float b2 = beta[i] * beta[i];
            x_out[i] = (uniform24(r[j]) < b2) ? 1 : 0;
            P += (int64_t)v[i] * x_out[i];
            W += (int64_t)w[i] * x_out[i];
        }
    }
    out[0] = (W <= cap) ? P : -(W - cap);
    out[1] = P;
    out[2] = W;
}

/* The same chromosome-local step with binary64 amplitudes (reading R8). */
void oracle_row_generation_f64(uint64_t seed, int64_t t, int64_t c, int64_t ng,
                               const int32_t *v, const int32_t *w, int64_t cap,
                               double *alpha, double *beta, const uint8_t *x_prev,
                               const uint8_t *elite_prev, int below_elite,
                               uint8_t *x_out, int64_t out[3])
{
    if (below_elite)
        for (int64_t i = 0; i < ng; ++i)
            if (x_prev[i] != elite_prev[i])
                oracle_cip_gene_f64(&alpha[i], &beta[i], elite_prev[i]);
    int64_t P = 0, W = 0;
    for (int64_t k = 0; 4 * k < ng; ++k) {
        uint32_t r[4];
        draws4(seed, t, c, k, r);
        for (int j = 0; j < 4 && 4 * k + j < ng; ++j) {
            const int64_t i = 4 * k + j;
            const double b2 = beta[i] * beta[i];
            const double u = (double)(r[j] >> 8) * 0x1p-24;
            x_out[i] = (u < b2) ? 1 : 0;
            P += (int64_t)v[i] * x_out[i];
            W += (int64_t)w[i] * x_out[i];
        }
    }
    out[0] = (W <= cap) ? P : -(W - cap);
    out[1] = P;
    out[2] = W;
}

/* Termination test of Sec. IV-A, read for integer fitness: the run has
 * converged after generation t when the elite fitness of the last `window`
 * generations (t-window+1 .. t) is one value (a spread within 1e-6 of the
 * mean means equality for integers). */
int oracle_converged(const oracle *s, int window)
{
    if (window < 1 || s->t < window || s->t > s->elite_cap) return 0;
    const int64_t last = s->elite_f[s->t - 1];
    for (int64_t k = s->t - window; k < s->t - 1; ++k)
        if (s->elite_f[k] != last) return 0;
    return 1;
}

/* Runs at most n more generations, stopping after the first generation at
 * which the run has converged (Fig. 1: terminate or next generation).
 * Returns the number of generations run by this call. */
int64_t oracle_run_until_converged(oracle *s, int64_t n, int window)
{
    int64_t g = 0;
    if (oracle_converged(s, window)) return 0;
    while (g < n) {
        oracle_generation(s);
        ++g;
        if (oracle_converged(s, window)) break;
    }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Accessors (copies into caller-owned buffers; any pointer may be NULL).   */
/* ------------------------------------------------------------------------ */
void oracle_get_amplitudes_f64(const oracle *s, double *alpha, double *beta)
{
    size_t n = (size_t)s->ng * (size_t)s->np;
    if (!s->f64) return;
    if (alpha) memcpy(alpha, s->alpha_d, n * sizeof(double));
    if (beta) memcpy(beta, s->beta_d, n * sizeof(double));
}

void oracle_set_amplitudes_f64(oracle *s, const double *alpha, const double *beta)
{
    size_t n = (size_t)s->ng * (size_t)s->np;
    if (!s->f64) return;
    if (alpha) memcpy(s->alpha_d, alpha, n * sizeof(double));
    if (beta) memcpy(s->beta_d, beta, n * sizeof(double));
}

void oracle_get_amplitudes(const oracle *s, float *alpha, float *beta)
{
    size_t n = (size_t)s->ng * (size_t)s->np;
    if (s->f64) return;
    if (alpha) memcpy(alpha, s->alpha, n * sizeof(float));
    if (beta) memcpy(beta, s->beta, n * sizeof(float));
}

void oracle_set_amplitudes(oracle *s, const float *alpha, const float *beta)
{
    size_t n = (size_t)s->ng * (size_t)s->np;
    if (s->f64) return;
    if (alpha) memcpy(s->alpha, alpha, n * sizeof(float));
    if (beta) memcpy(s->beta, beta, n * sizeof(float));
}

/* Rows [row0, row0 + n) of the amplitudes, in the oracle's precision
 * (float or double arrays of n * ng), and of the alleles; any pointer may be
 * NULL.  Rows outside the population are not copied. */
void oracle_get_rows(const oracle *s, int64_t row0, int64_t n, void *alpha, void *beta,
                     uint8_t *x)
{
    if (row0 < 0 || n < 0 || row0 + n > s->np) return;
    const size_t off = (size_t)row0 * (size_t)s->ng, cnt = (size_t)n * (size_t)s->ng;
    const size_t el = s->f64 ? sizeof(double) : sizeof(float);
    const char *a = s->f64 ? (const char *)s->alpha_d : (const char *)s->alpha;
    const char *b = s->f64 ? (const char *)s->beta_d : (const char *)s->beta;
    if (alpha) memcpy(alpha, a + off * el, cnt * el);
    if (beta) memcpy(beta, b + off * el, cnt * el);
    if (x) memcpy(x, s->x + off, cnt);
}

void oracle_get_alleles(const oracle *s, uint8_t *x)
{
    memcpy(x, s->x, (size_t)s->ng * (size_t)s->np);
}

void oracle_set_alleles(oracle *s, const uint8_t *x)
{
    memcpy(s->x, x, (size_t)s->ng * (size_t)s->np);
}

void oracle_get_fitness(const oracle *s, int64_t *fit, int64_t *P, int64_t *W)
{
    if (fit) memcpy(fit, s->fit, sizeof(int64_t) * s->np);
    if (P) memcpy(P, s->P, sizeof(int64_t) * s->np);
    if (W) memcpy(W, s->W, sizeof(int64_t) * s->np);
}

void oracle_set_fitness(oracle *s, const int64_t *fit)
{
    memcpy(s->fit, fit, sizeof(int64_t) * s->np);
}

int64_t oracle_generation_index(const oracle *s) { return s->t; }
int64_t oracle_elite(const oracle *s) { return s->elite; }

/* best: {has_best, f, P, W, generation, chromosome}; bits: ng bytes or NULL */
void oracle_get_best(const oracle *s, int64_t out[6], uint8_t *bits)
{
    out[0] = s->has_best; out[1] = s->best_f; out[2] = s->best_P;
    out[3] = s->best_W; out[4] = s->best_gen; out[5] = s->best_chrom;
    if (bits) memcpy(bits, s->best_x, (size_t)s->ng);
}
