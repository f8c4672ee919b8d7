/*
 * libqieo -- quantum-inspired evolutionary optimization (QIEO) of the 0/1
 * knapsack problem on one AMD Instinct MI355X (gfx950).
 *
 * The library runs the per-generation loop of the paper (Srikanth et al.,
 * "Evaluation of portability and performance of an OpenMP5 offloaded
 * Quantum-Inspired Evolutionary Optimization Across the GPU Ecosystem"):
 * QIP observes every qubit gene, Evaluation scores every chromosome with the
 * knapsack fitness of eq. (1), DetermineElite picks the generation best, and
 * CIP rotates every qubit toward that elite (Sec. III-B, Fig. 1).  All four
 * steps run on the GPU; the population stays resident in device memory.
 *
 * Conventions for every call:
 *   - Return value 0 (QIEO_OK) on success, a negative QIEO_E* code otherwise;
 *     qieo_last_error() then holds a thread-local message.  No C++ exception
 *     crosses this interface.
 *   - Every input array is host memory and is copied; the caller keeps
 *     ownership.  Every output array is caller-owned host memory of the stated
 *     length.  Handles are owned by the caller until the matching destroy.
 *   - One thread at a time per handle; distinct handles are independent.
 *   - A run is deterministic: the state after qieo_step(h, a) followed by
 *     qieo_step(h, b) equals the state after qieo_step(h, a + b), and equals
 *     the same instance run alone, in a batch, or inside the server.
 *
 * Readings of points the paper leaves open (the CPU oracle implements the
 * same ones):
 *   - allele 1 is observed iff u < beta^2, with u the 24-bit uniform
 *     (r >> 8) * 2^-24 of the 32-bit Philox4x32-10 word r drawn with counter
 *     {gene/4, chromosome, generation, 0} and key {seed lo, seed hi}; gene i
 *     takes word i mod 4;
 *   - amplitudes are binary32, initialised to fl32(1/sqrt 2); fitness is exact
 *     int32 with penalty factor lambda = 1 (any lambda > 0 gives the same run);
 *   - the elite is the generation best, lowest index on ties; chromosome c
 *     rotates gene i only when f(c) < f(elite) and x[c][i] differs from the
 *     elite's allele, by 0.01*pi toward it, then one Newton step
 *     g = 1.5 - 0.5*(a^2 + b^2) rescales (a, b) toward unit norm.
 */
#ifndef QIEO_H
#define QIEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define QIEO_OK         0
#define QIEO_EINVAL    -1   /* bad argument: sizes, null pointers, ranges      */
#define QIEO_EOVERFLOW -2   /* sum of values or weights exceeds INT32_MAX      */
#define QIEO_ENOMEM    -3   /* device (or host) allocation failed / no room    */
#define QIEO_EDEVICE   -4   /* HIP runtime error or no usable gfx950 device    */
#define QIEO_EAGAIN    -5   /* result not ready yet (server poll)              */
#define QIEO_ESTATE    -6   /* call not valid in the object's current state   */

/* ---- problem description (Sec. III-A) ----------------------------------- */
/* Item i of the knapsack: value v_i (profit) and weight w_i, both >= 0. */
typedef struct qieo_item {
    int32_t profit;
    int32_t weight;
} qieo_item;

/* Best chromosome found so far (the best generation elite).  fitness follows
 * eq. (1) with lambda = 1: the profit when weight <= capacity, otherwise
 * -(weight - capacity).  generation is the index (from 0) of the generation
 * that first produced it, chromosome its row in that generation.
 * generation = -1 when no generation has run yet. */
typedef struct qieo_result {
    int32_t fitness;
    int32_t profit;
    int32_t weight;
    int32_t feasible;
    int64_t generation;
    int64_t chromosome;
} qieo_result;

/* Optional device context.  alloc/free replace hipMalloc/hipFree for the
 * instance's device memory (both NULL: hipMalloc/hipFree); alloc returns NULL
 * on failure.  stream is a hipStream_t on which all work is ordered (NULL:
 * the library creates and owns one stream per handle). */
typedef struct qieo_dev_ctx {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
    void *stream;
} qieo_dev_ctx;

typedef struct qieo_inst qieo_inst;

/* ---- single instance ----------------------------------------------------- */

/* Creates one population of n_pop chromosomes of n_items qubit genes for the
 * knapsack (items, capacity) (Sec. III-A) and initialises every amplitude pair
 * on the device.  Requires n_items >= 1, n_pop >= 1, capacity >= 0, every
 * profit and weight >= 0, n_items <= 2^30 - 256 and n_pop times n_items
 * rounded up to 64 at most 2^36 genes (QIEO_EINVAL), and sum(profit),
 * sum(weight) <= INT32_MAX (QIEO_EOVERFLOW).  seed keys the Philox draws.  On success *out
 * receives the handle; on failure nothing is allocated. */
int qieo_create(const qieo_item *items, int32_t n_items, int32_t capacity,
                int32_t n_pop, uint64_t seed, qieo_inst **out);

/* As qieo_create, with an optional device context (NULL = defaults). */
int qieo_create_ex(const qieo_item *items, int32_t n_items, int32_t capacity,
                   int32_t n_pop, uint64_t seed, const qieo_dev_ctx *ctx,
                   qieo_inst **out);

/* As qieo_create_ex with binary64 amplitudes (the paper's precision, Sec. V):
 * the same steps with binary64 roundings of the same constants (cos and sin
 * of 0.01 pi, 1/sqrt 2); the uniform draws are unchanged.  Twice the
 * amplitude memory and traffic.  Such an instance runs the fused pipeline with
 * per-generation launches; its amplitudes are read with
 * qieo_export_rows_f64. */
int qieo_create_f64(const qieo_item *items, int32_t n_items, int32_t capacity,
                    int32_t n_pop, uint64_t seed, const qieo_dev_ctx *ctx, qieo_inst **out);

/* Runs n_generations full generations (QIP, Evaluation, DetermineElite, CIP;
 * Sec. III-B, Fig. 1) and waits for them.  n_generations >= 0. */
int qieo_step(qieo_inst *h, int32_t n_generations);

/* As qieo_step, without waiting: the work is queued on the handle's stream.
 * Host-side reads of the handle (qieo_best, export) wait by themselves. */
int qieo_step_async(qieo_inst *h, int32_t n_generations);

/* Waits for all queued work of the handle. */
int qieo_sync(qieo_inst *h);

/* Best-so-far chromosome.  bits_or_null, if not NULL, receives the allele
 * string packed little-endian (item i is bit i%32 of word i/32); n_words must
 * be >= ceil(n_items/32) (QIEO_EINVAL otherwise). */
int qieo_best(qieo_inst *h, qieo_result *out, uint32_t *bits_or_null,
              size_t n_words);

/* qieo_best for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it.  Same arguments and results as qieo_best; it calls no
 * hipMalloc, hipFree or other allocating routine (on success it allocates no
 * host memory either).  The best string is unpacked on the device into a static
 * staging buffer of the library (QIEO_BEST_NOALLOC_MAX_ITEMS genes, 1 MiB,
 * one per device, held until the process ends) and copied from there into
 * bits_or_null.  Every call on a device shares that buffer: calls that
 * overlap on one device (from different threads, or with streams not
 * ordered against each other) race and must be serialised by the caller.
 * With bits_or_null != NULL, an instance of more than
 * QIEO_BEST_NOALLOC_MAX_ITEMS items gives QIEO_EINVAL (use qieo_best). */
#define QIEO_BEST_NOALLOC_MAX_ITEMS (1 << 23)
int qieo_best_noalloc(qieo_inst *h, qieo_result *out, uint32_t *bits_or_null, size_t n_words);

/* Number of generations run so far (waits for queued work). */
int qieo_generations(qieo_inst *h, int64_t *out);

/* Termination by convergence (Sec. IV-A: the elite fitness is stable for a
 * window of generations).  With window w in [1, 32], the run stops after the
 * first generation t whose elite fitness equals that of generations
 * t-w+1 .. t-1; later qieo_step calls run nothing.  0 (default) keeps fixed
 * budgets.  Must be set before the first generation (QIEO_ESTATE). */
int qieo_set_convergence(qieo_inst *h, int32_t window);
/* converged = 1 once the window test has fired; generation = the generation
 * after which it stopped (-1 if not converged). */
int qieo_converged(qieo_inst *h, int32_t *converged, int64_t *generation);

/* Copies rows [row0, row0 + n_rows) of the population state after the last
 * completed generation t-1, with that generation's CIP applied, to host
 * arrays (row-major, n_items per row): alpha, beta (binary32 amplitudes),
 * alleles (0/1 bytes observed at t-1), and for each row fitness, profit and
 * weight at t-1.  Any pointer may be NULL.  elite (may be NULL) receives the
 * elite index of generation t-1, or -1 when no generation has run.  The
 * device state is not modified.  Requires 0 <= row0, n_rows >= 0,
 * row0 + n_rows <= n_pop. */
int qieo_export_rows(qieo_inst *h, int32_t row0, int32_t n_rows,
                     float *alpha, float *beta, uint8_t *alleles,
                     int32_t *fitness, int32_t *profit, int32_t *weight,
                     int32_t *elite);

/* Checkpoint and resume of the whole state between two generations (the
 * population Q of Fig. 1, the generation counter, the best-so-far record and
 * the convergence history).  qieo_state_size gives the bytes of a snapshot;
 * qieo_export_state writes one into a caller-owned host buffer of at least
 * that size: a versioned header (problem shape, seed, a hash of the items,
 * precision, generations done) followed by the device state, including the
 * last generation's rotation still pending.  qieo_import_state loads a
 * snapshot into a handle created with the same items, capacity, n_pop, seed
 * and precision (its own earlier state is replaced); the handle then
 * continues the trajectory bit for bit as if it had run the exported
 * generations itself.  A snapshot of another problem, precision or version,
 * or a short buffer, gives QIEO_EINVAL and leaves the handle unchanged; a
 * snapshot with a convergence window needs the fused pipeline (QIEO_ESTATE).
 * Both wait for the handle's stream. */
int qieo_state_size(qieo_inst *h, size_t *bytes);
int qieo_export_state(qieo_inst *h, void *buf, size_t bytes);
int qieo_import_state(qieo_inst *h, const void *buf, size_t bytes);

/* qieo_export_rows for a binary64 instance (alpha, beta as doubles). */
int qieo_export_rows_f64(qieo_inst *h, int32_t row0, int32_t n_rows,
                         double *alpha, double *beta, uint8_t *alleles,
                         int32_t *fitness, int32_t *profit, int32_t *weight,
                         int32_t *elite);

/* Releases the handle and all its device memory (NULL is ignored). */
void qieo_destroy(qieo_inst *h);

/* Work shape of the generation kernel for this handle: rows_per_block in
 * {1, 2, 4} chromosomes per workgroup, waves_per_block in [1, 16] wavefronts
 * splitting each chromosome's genes.  0 for either keeps the library's
 * choice.  The shape changes speed only, never results.  Out-of-range values
 * give QIEO_EINVAL. */
int qieo_set_tile(qieo_inst *h, int32_t rows_per_block, int32_t waves_per_block);
/* Current work shape. */
int qieo_get_tile(qieo_inst *h, int32_t *rows_per_block, int32_t *waves_per_block);
/* Code variant of the generation kernel, a set of bits in [0, 31]: bit 0
 * prefetches the next chunk's amplitudes while the current one is computed,
 * bit 1 stores amplitudes with non-temporal hints, bit 2 loads them with
 * non-temporal hints, bit 3 re-derives the previous generation's alleles
 * from the stored beta and their draws instead of reading the stored allele
 * words back, bit 4 runs each generation in segment order (one workgroup per
 * 1024-gene segment of a row, each of the device's XCDs sweeping one
 * contiguous run of segments in address order, then a small launch
 * closing the rows' sums; the work shape of qieo_set_tile does not apply;
 * bit 0 is ignored).  Binary64 handles ignore bit 3 in row order.  Variants
 * change speed only, never results.  Out-of-range values give QIEO_EINVAL. */
int qieo_set_kernel_flags(qieo_inst *h, int32_t flags);
/* Current variant bits (the library's choice until qieo_set_kernel_flags). */
int qieo_get_kernel_flags(qieo_inst *h, int32_t *flags);

/* ---- batch: many instances advanced together (one device pool) ---------- */

/* One knapsack problem plus its QIEO parameters (Sec. III-A): items as for
 * qieo_create, capacity, population size n_pop, Philox seed. */
typedef struct qieo_problem {
    const qieo_item *items;
    int32_t n_items;
    int32_t capacity;
    int32_t n_pop;
    uint64_t seed;
} qieo_problem;

typedef struct qieo_batch qieo_batch;

/* Creates n >= 1 populations, each exactly as qieo_create would, in one
 * device pool of the summed size.  Each problem is validated as in
 * qieo_create (the failing index is named in qieo_last_error()).  Instances
 * are numbered 0..n-1 in input order. */
int qieo_batch_create(const qieo_problem *probs, int32_t n, const qieo_dev_ctx *ctx,
                      qieo_batch **out);

/* Runs n_gen_per_inst[i] >= 0 generations of instance i, for every i (array
 * of qieo_batch_size entries), all instances in the same launches; waits.
 * Each instance's state afterwards is bit-identical to running it alone with
 * qieo_step. */
int qieo_batch_step(qieo_batch *b, const int32_t *n_gen_per_inst);
/* As qieo_batch_step without waiting; the counts are copied before return. */
int qieo_batch_step_async(qieo_batch *b, const int32_t *n_gen_per_inst);
int qieo_batch_sync(qieo_batch *b);
int qieo_batch_size(const qieo_batch *b, int32_t *n);
int qieo_batch_generations(qieo_batch *b, int32_t i, int64_t *out);
/* Best-so-far of instance i; bits as for qieo_best. */
int qieo_batch_best(qieo_batch *b, int32_t i, qieo_result *out, uint32_t *bits,
                    size_t n_words);
/* Row export of instance i, as qieo_export_rows. */
int qieo_batch_export_rows(qieo_batch *b, int32_t i, int32_t row0, int32_t n_rows,
                           float *alpha, float *beta, uint8_t *alleles, int32_t *fitness,
                           int32_t *profit, int32_t *weight, int32_t *elite);
/* Convergence window for every instance of the batch (see qieo_set_convergence). */
int qieo_batch_set_convergence(qieo_batch *b, int32_t window);
int qieo_batch_converged(qieo_batch *b, int32_t i, int32_t *converged, int64_t *generation);
/* Work shape for every launch of the batch (rows_per_block = 0 restores the
 * library's per-class choice); see qieo_set_tile and qieo_set_kernel_flags
 * (bit 4, segment order, is for single instances: QIEO_EINVAL here). */
int qieo_batch_set_tile(qieo_batch *b, int32_t rows_per_block, int32_t waves_per_block,
                        int32_t flags);
/* 1 (default): a call that repeats the previous one (same longest
 * generation count, no membership change in between) is captured into a HIP
 * graph, which later such calls replay; a one-off call is launched directly.
 * 0: always launched one by one.  A capture that another thread's
 * device-wide call invalidates falls back to direct launches.  Results are
 * identical. */
int qieo_batch_set_graph(qieo_batch *b, int32_t enabled);
/* 1 (default): members whose whole state fits in one workgroup's LDS (see
 * qieo_set_persistent, mode 1) run as one workgroup each for the whole call,
 * concurrently with the per-generation launches of the others; 0: all
 * members use per-generation launches.  Results are identical. */
int qieo_batch_set_persistent(qieo_batch *b, int32_t enabled);
/* 1 (default): when the batch's amplitude planes exceed 256 MB, members with
 * rows of 8 or more 256-gene chunks run in segment order (see
 * qieo_set_kernel_flags, bit 4), all of them in one launch over a table of
 * 1024-gene segments in address order, plus one launch closing their rows,
 * as long as that table stays within 4M segments (4.3e9 genes); if it would
 * not, the members with rows of 32 or more chunks alone, under the same
 * limit.  2: the members with rows of 32 or more chunks only.  0: row order
 * for every member.  Other values give QIEO_EINVAL.  Ignored while
 * qieo_batch_set_tile forces a shape.  Results are identical. */
int qieo_batch_set_segment_order(qieo_batch *b, int32_t mode);
/* 1 (default): every member that fits runs every generation of a call
 * inside cooperative launches with its amplitude planes held in registers,
 * the on-chip loop of qieo_set_persistent mode 3 extended to many members:
 * each member on workgroups of whole rows (rows of up to 76 chunks of 256
 * genes, 146 when every profit and weight is below 2^14: the member's item
 * tables and two generations of its rows' allele words must fit a
 * workgroup's LDS), its workgroups waiting only for each other at the end
 * of each
 * generation (Sec. III-B's loop: DetermineElite over the member's rows
 * before its CIP), at most one workgroup per CU, so a batch of more rows
 * than that takes several such launches one after another; they run before
 * the call's other launches, alone on the device.  The members it cannot
 * place (longer rows, too many rows for one launch) keep the per-generation
 * launches (LDS-resident, segment or row order as set above).  Members with
 * a convergence window (qieo_batch_set_convergence) run in launches of their
 * own that make the window test (every workgroup of a member stops at the
 * generation the per-generation launches would).  Not taken while a shape
 * is forced, nor with graph capture (such a call is launched directly).  0: every member
 * per-generation launches.  Results are identical.  A barrier wait past its
 * bound (qieo_batch_set_barrier_timeout) makes the call fail with
 * QIEO_EDEVICE when the batch is synchronised, its members' state then
 * undefined. */
int qieo_batch_set_onchip(qieo_batch *b, int32_t enabled);
/* On-chip launches (see qieo_batch_set_onchip) one call of the current
 * membership makes (0 if none); plans the batch if membership changed. */
int qieo_batch_onchip_launches(qieo_batch *b, int32_t *n);
/* Bound on one barrier wait of the batched on-chip loop, in microseconds
 * (default one second); QIEO_EINVAL if negative. */
int qieo_batch_set_barrier_timeout(qieo_batch *b, int64_t microseconds);
void qieo_batch_destroy(qieo_batch *b);

/* ---- server: continuous batching of solve requests ----------------------- */

/* hbm_budget_bytes: size of the device pool that holds resident populations
 * (one allocation at create; a request is admitted only when its population
 * fits).  max_resident: cap on concurrently resident requests (0 = none).
 * gens_per_iter: generations every resident population advances per engine
 * iteration (0 = 25); admissions and retirements happen between iterations. */
typedef struct qieo_server_cfg {
    size_t hbm_budget_bytes;
    int32_t max_resident;
    int32_t gens_per_iter;
    int32_t convergence_window;   /* as qieo_set_convergence, for every request (0 = off) */
} qieo_server_cfg;

typedef struct qieo_server_stats {
    int64_t queued, resident, admitted, completed, failed, iterations;
    double gene_updates;          /* sum of Np*Ng*generations run so far */
    size_t pool_bytes, pool_used;
    int64_t peak_resident;
    size_t peak_pool_used;
    int32_t error;                /* first worker error (0 = none) */
} qieo_server_stats;

typedef struct qieo_server qieo_server;

/* Creates the server and its worker thread (which owns all GPU work). */
int qieo_server_create(const qieo_server_cfg *cfg, const qieo_dev_ctx *ctx, qieo_server **out);
/* Queues a request to run n_gen >= 1 generations of a fresh population for
 * problem p (copied; validated as in qieo_create).  Thread-safe.  *ticket
 * identifies it.  Its result is bit-identical to qieo_create + qieo_step(n_gen)
 * + qieo_best on the same inputs, whatever else is resident. */
int qieo_server_submit(qieo_server *s, const qieo_problem *p, int32_t n_gen, uint64_t *ticket);
/* 1 (default): the residents' generations run in batched on-chip launches
 * wherever they fit (see qieo_batch_set_onchip), the rest in per-generation
 * launches; 0: per-generation launches only.  Takes effect at the worker's
 * next iteration.  Results are identical. */
int qieo_server_set_onchip(qieo_server *s, int32_t enabled);
/* QIEO_EAGAIN while the request is queued or running; otherwise its result
 * (or its failure code, e.g. QIEO_ENOMEM when its population can never fit
 * the budget).  latency_ns = completion - submission, steady clock. */
int qieo_server_poll(qieo_server *s, uint64_t ticket, qieo_result *out, uint32_t *bits,
                     size_t n_words, int64_t *latency_ns);
/* As qieo_server_poll, blocking until the request has finished. */
int qieo_server_wait(qieo_server *s, uint64_t ticket, qieo_result *out, uint32_t *bits,
                     size_t n_words, int64_t *latency_ns);
/* Forgets a finished request (its result can no longer be polled). */
int qieo_server_release(qieo_server *s, uint64_t ticket);
int qieo_server_get_stats(qieo_server *s, qieo_server_stats *out);
/* Stops the worker after its current iteration and frees everything. */
void qieo_server_destroy(qieo_server *s);

/* Whole-call launches (binary32, fused pipeline).  One launch runs all
 * generations of a qieo_step call, barriers replacing launch boundaries:
 *  - single workgroup: the whole state (amplitudes, allele words, item
 *    tables, fitness) in one workgroup's LDS, or read from global memory;
 *  - on-chip grid: one cooperative launch, one workgroup per compute unit,
 *    the amplitude planes held in registers for the call and written back
 *    at its end, a grid barrier per generation (Sec. III-B's loop, with
 *    DetermineElite's result final at each barrier).  It takes populations
 *    of up to 16 x 10 (row, 256-gene chunk) items per compute unit whose
 *    item tables fit in LDS, e.g. 1024 x 10,000 on 256 compute units,
 *    with or without a convergence window (each workgroup makes the window
 *    test on the elites it gathers; all stop at the same generation).
 * mode 0: never (per-generation launches); 1 (default): the single
 * workgroup from LDS for tiny populations (n_pop * ceil(n_items / 256) <=
 * 16), the on-chip grid for calls of >= 4 generations of populations it
 * takes that have n_pop >= 256, n_pop * ceil(n_items / 256) >= 1024 or
 * n_items > 4864 (rows of 20 chunks), where it measured faster than
 * launches; 2: a
 * single workgroup whenever the state fits in LDS, else from
 * global memory when n_pop <= 2048; 3: the on-chip grid for every call it
 * takes.  A population or call a mode does not take runs as mode 0.
 * Results are identical in every mode.  On-chip launches of different
 * instances on one device run one after another, whatever their streams
 * (each grid holds every CU).  An on-chip grid barrier that waits
 * longer than its bound (qieo_set_barrier_timeout, default one second) ends
 * the launch; qieo_sync then reports QIEO_EDEVICE and the instance's state
 * is undefined. */
int qieo_set_persistent(qieo_inst *h, int32_t mode);
/* How the last qieo_step[_async] call ran: QIEO_PATH_LAUNCHES (a launch
 * per generation, or per step of the unfused pipelines), QIEO_PATH_LDS (one
 * single-workgroup launch from LDS), QIEO_PATH_GLOBAL (one single-workgroup
 * launch from global memory), QIEO_PATH_ONCHIP (one on-chip grid launch);
 * -1 before the first call. */
#define QIEO_PATH_LAUNCHES 0
#define QIEO_PATH_LDS 1
#define QIEO_PATH_GLOBAL 2
#define QIEO_PATH_ONCHIP 3
int qieo_get_call_path(qieo_inst *h, int32_t *path);
/* Bound on one grid-barrier wait of the on-chip loop, in microseconds of the
 * device's wall clock (a watchdog: a generation takes tens of microseconds);
 * [0, 3600 s], default 1 s. */
int qieo_set_barrier_timeout(qieo_inst *h, int64_t microseconds);

/* 1 (default): a qieo_step call of n >= 2 generations on the fused
 * per-generation path that repeats the previous call (same n, work shape and
 * variant) is captured into a HIP graph (n launches plus the finishing one),
 * which later calls with the same n and shape replay; a one-off call is
 * launched directly.  0: always launched one by one.  Timing mode always
 * launches one by one.  If another thread's device-wide call invalidates a
 * capture in progress, that call's launches are enqueued directly.  Results
 * are identical in every case. */
int qieo_set_graph(qieo_inst *h, int32_t enabled);

/* ---- work-shape autotuner ------------------------------------------------ */

typedef struct qieo_tune_result {
    int32_t rows_per_block, waves_per_block, flags;
    int32_t candidates;                 /* shapes timed */
    double ms_per_generation;           /* of the chosen shape */
    double worst_ms_per_generation;     /* of the slowest candidate */
} qieo_tune_result;

/* Times every work shape (rows per workgroup 1/2/4 x waves 2/4/8/16, waves
 * not above the chunks per row, x the sixteen row-order sets of variant bits
 * 0-3; plus segment order under each of its four cache-hint settings) for
 * trial_generations generations each on a scratch population of n_pop x
 * n_items (its own device memory, twice the population's, freed before
 * return; items NULL = items like the workloads': weights uniform in
 * [1, 100], value = weight + 10, capacity half the weight sum).  Every
 * candidate runs the same generations from the same state (a copy of the
 * scratch population after two warm-up generations, restored before each
 * candidate), twice, in opposite orders; the faster time counts.  Records
 * the fastest in the tuning database under the shape's bucket (log2 of
 * n_pop, log2 of 256-gene chunks per row) and returns it.  Later qieo_create
 * calls whose shape falls in a tuned bucket use that shape.  A shape
 * qieo_create would reject, or trial_generations outside [1, 1000], gives
 * QIEO_EINVAL before any allocation; QIEO_ENOMEM if the scratch population
 * does not fit in device memory. */
int qieo_autotune(int32_t n_items, int32_t n_pop, const qieo_item *items, int32_t capacity,
                  int32_t trial_generations, qieo_tune_result *out);

/* One launch class of a batch (members grouped by 256-gene chunks per row:
 * class 0 = 1 chunk, 1 = 2-3, 2 = 4-7, 3 = 8-31, 4 = 32 or more; a batch
 * whose planes exceed 256 MB runs its classes 3 and 4 together in segment
 * order, as class 4) as timed by qieo_batch_autotune. */
typedef struct qieo_class_tune {
    int32_t shape_class;
    int32_t rows;                       /* chromosomes in the class */
    int32_t max_chunks;                 /* its longest row, in 256-gene chunks */
    int32_t rows_per_block, waves_per_block, flags;   /* the chosen shape */
    int32_t default_rows_per_block, default_waves_per_block, default_flags;
    int32_t candidates;                 /* shapes timed */
    double ms_per_generation;           /* the chosen shape's, the class alone */
    double default_ms_per_generation;   /* the built-in rule's shape, the class alone */
} qieo_class_tune;

/* Tunes the work shape of every launch class of batch b on the batch itself:
 * per class, row order with rows per workgroup 1/2/4 x waves per workgroup
 * half, equal to and twice the class's default x variant bits 0-2, and for
 * the long-row class of a batch whose planes exceed 256 MB segment order
 * under its four cache-hint settings; each candidate runs trial_generations
 * generations of that class alone, from the same state (the members' state
 * is saved first and restored before every candidate and at the end: the
 * batch's trajectory does not move), twice in opposite orders, the faster
 * time counting.  Records each class's fastest shape in the tuning database
 * (bucket: class, log2 of its rows, log2 of its longest row) and rebuilds
 * the batch's classes with them; later batches and servers whose classes
 * fall in a tuned bucket use them too.  out (may be NULL) receives up to
 * max_out entries, *n_out (may be NULL) the number of classes.  Needs device
 * memory for a copy of the members' state (QIEO_ENOMEM otherwise);
 * trial_generations outside [1, 1000] gives QIEO_EINVAL.  Results of later
 * calls are unchanged (work shapes never change results).
 * A batch with on-chip launches (qieo_batch_set_onchip) also gets its
 * items-per-wave variants tuned: every subset of the usable variants
 * K = 2, 4, 6, 8, 10 that holds the largest is planned for the members
 * the current plan places on-chip and timed with all its launches for
 * trial_generations generations from the same state (twice, in opposite
 * orders); the fastest subset is kept for this batch's later calls,
 * recorded in the tuning database as class -1 (bucket: log2 of all the
 * batch's rows, log2 of its longest row; later batches and servers in the
 * bucket use it) and reported as an entry with shape_class -1:
 * rows and max_chunks of the on-chip members, flags = the chosen subset
 * (bit v: K = 2v + 2), rows_per_block = its launches per call,
 * waves_per_block = 16, the default_* fields the same for the subset in
 * use before, candidates = subsets timed, ms_per_generation for all the
 * launches together. */
int qieo_batch_autotune(qieo_batch *b, int32_t trial_generations, qieo_class_tune *out,
                        int32_t max_out, int32_t *n_out);
/* Tuning database as JSON (one entry per line, single-instance buckets and
 * batch classes); load returns the number of entries read (>= 0) or a
 * negative status. */
int qieo_tune_db_save(const char *path);
int qieo_tune_db_load(const char *path);
void qieo_tune_db_clear(void);

/* ---- pipeline variants (the paper's four-region structure) -------------- */

/* QIEO_PIPELINE_FUSED (default): one launch per generation.
 * QIEO_PIPELINE_UNFUSED: per generation CIP, QIP and Evaluation as three
 *   launches and DetermineElite as a fourth (the four timed regions of eq. (2),
 *   Sec. III-B).
 * QIEO_PIPELINE_UNFUSED_FE_DE: DetermineElite fused into Evaluation's last
 *   write (Sec. VI, P4, second option).
 * QIEO_PIPELINE_UNFUSED_HOST_DE: DetermineElite on the host: fitness copied
 *   out, argmax on the CPU, elite copied back, every generation (Sec. VI, P4,
 *   first option).
 * QIEO_PIPELINE_CHROMOSOME: the chromosome-parallel mapping of eq. (3): one
 *   GPU lane per chromosome walks its genes serially (fused steps).
 * All variants give bit-identical results; they exist to measure the cost of
 * each step and of the mapping.  Only the default runs the convergence test. */
#define QIEO_PIPELINE_FUSED 0
#define QIEO_PIPELINE_UNFUSED 1
#define QIEO_PIPELINE_UNFUSED_FE_DE 2
#define QIEO_PIPELINE_UNFUSED_HOST_DE 3
#define QIEO_PIPELINE_CHROMOSOME 4
int qieo_set_pipeline(qieo_inst *h, int32_t pipeline);
/* With timing enabled: per stage {fused generation, CIP, QIP, Evaluation,
 * DetermineElite} the number of timed launches (host DetermineElite: timed
 * sections) and their summed milliseconds (arrays of 5). */
int qieo_stage_time(qieo_inst *h, int64_t *launches, double *total_ms, int reset);

/* ---- errors and introspection ------------------------------------------- */
const char *qieo_strerror(int code);
/* Message of the last failing call on this thread ("" if none). */
const char *qieo_last_error(void);
/* Library version string. */
const char *qieo_version(void);

/* Kernel timing, for measurement.  When enabled, the library records HIP
 * events on the handle's stream around every generation kernel it launches;
 * qieo_kernel_time returns the number of such launches and their summed
 * duration in milliseconds since the last reset, and resets on request.
 * Timing adds two event records per generation. */
int qieo_set_timing(qieo_inst *h, int enabled);
int qieo_kernel_time(qieo_inst *h, int64_t *launches, double *total_ms, int reset);

#ifdef __cplusplus
}
#endif
#endif /* QIEO_H */
