/*
 * pamc.h -- population annealing Monte Carlo for Edwards-Anderson spin
 * glasses in 3D (+-J or real, e.g. Gaussian, couplings) and 2D (real
 * couplings) on AMD Instinct MI355X (gfx950).
 *
 * The operation is the one of Barzegar, Pattison, Wang and Katzgraber,
 * "Optimization of population annealing Monte Carlo for large-scale
 * spin-glass simulations" (arXiv:1710.09025):
 *   - Sec. II.A, Eq. (1): H = -sum_<ij> J_ij S_i S_j on the periodic L^D
 *     lattice, N = L^D Ising spins (D = 3, or D = 2 through
 *     pamc_options.dim), couplings J_ij = +-1 (pamc_create, D = 3) or real
 *     (pamc_create_real: the paper's Gaussian case study, held in fixed
 *     point, J = j 2^-20 with int32 j, |J| < 8);
 *   - Sec. II.B: R replicas start at random at beta_0 = 0; at each of the
 *     n_temps inverse temperatures beta_k the library runs `sweeps`
 *     Metropolis sweeps on every replica (one sweep = N attempted flips,
 *     checkerboard order of Sec. III.A), measures, and resamples to
 *     beta_{k+1}: replica i gets floor(tau_i) or ceil(tau_i) copies with
 *     tau_i = R exp(-(beta_{k+1}-beta_k) E_i) / sum_j exp(...), so the
 *     expected population stays R;
 *   - Sec. II.B, Eq. (2), Sec. V.A, Eq. (9): per-step observables (mean
 *     energy, specific heat, free energy by free-energy perturbation, family
 *     entropy S_f, entropic family size rho_s) and, at selected steps, the
 *     spin-overlap histogram.
 *
 * Every random number is a Philox4x32-10 word keyed by the run's seed and
 * counted by (site, replica row, step, sweep), so every output is a pure
 * function of (L, couplings, R, beta, sweeps, seed): it does not depend on
 * options, spin format, launch shapes, streams or batch composition.
 *
 * Conventions for every call:
 *   - all pointers are host pointers unless stated otherwise;
 *   - inputs are copied, the caller keeps ownership of its buffers;
 *   - outputs go to caller-owned host buffers of the stated size;
 *   - every call returns a status (PAMC_OK or a negative PAMC_ERR_*); none
 *     aborts or throws; pamc_last_error() gives a message for the calling
 *     thread;
 *   - a failed call leaves the handle as it was, except PAMC_ERR_DEVICE,
 *     after which the handle only accepts pamc_destroy().
 * A handle is used by one thread at a time.
 */
#ifndef PAMC_H
#define PAMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PAMC_OK = 0,
    PAMC_ERR_INVALID = -1,  /* an argument is out of range                  */
    PAMC_ERR_NOMEM = -2,    /* a device or host allocation failed           */
    PAMC_ERR_CAPACITY = -3, /* resampling would exceed the capacity         */
    PAMC_ERR_EXTINCT = -4,  /* resampling produced an empty population      */
    PAMC_ERR_DEVICE = -5,   /* a HIP call failed; the handle is poisoned     */
    PAMC_ERR_STATE = -6,    /* the call does not fit the handle's state     */
    PAMC_ERR_BUSY = -7,     /* the request or handle is not finished        */
    PAMC_ERR_REJECTED = -8  /* a serving request can never fit the budget   */
};

/* Spin storage on the device. */
enum { PAMC_SPINS_INT8 = 0, PAMC_SPINS_PACKED = 1 };

typedef struct pamc_options {
    int spin_format;         /* spin buffers in HBM: PAMC_SPINS_INT8 (default),
                                one byte per site, or PAMC_SPINS_PACKED, one
                                bit per site (rows 8x smaller; the sweeps
                                expand a tile to bytes on chip and pack it
                                when they write it back).  Results are
                                identical for both                          */
    int64_t capacity;        /* rows reserved per buffer; 0 = R + ceil(8 sqrt R) + 64 */
    void *stream;            /* hipStream_t to run on; NULL = a library stream  */
    /* optional device allocator (e.g. a framework's caching allocator):
     * alloc(bytes, user) returns device memory or NULL; free(ptr, user). */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *alloc_user;
    const int32_t *overlap_steps; /* steps at which to histogram the overlap; */
    int n_overlap_steps;          /* NULL/0 = only the last step             */
    int fuse_gather;         /* 1 (default): the next sweep reads surviving rows
                                through the copy map; 0: a separate gather
                                kernel copies them first (same results)      */
    int device;              /* HIP device ordinal; -1 = current device       */
    int tile_rows;           /* replica rows per sweep workgroup; 0 = the
                                library's choice for the lattice size; for
                                L = 8 and 16 rounded up to a multiple of the
                                replicas one pass sweeps (any value gives
                                identical results)                           */
    int graphs;              /* 1 (default): capture one temperature step in
                                a hipGraph and replay it for every step (not
                                with timing = 1); 0: launch kernels directly */
    int timing;              /* 1: record HIP events around the sweep and the
                                resampling kernels of every step (see
                                pamc_phase_times); 0 (default): no events   */
    int group_replicas;      /* L other than 8 and 16 (colour-major sweep):
                                replicas one sweep workgroup holds at once,
                                a multiple of four (they are swept in
                                fours); 0 = the library's choice.  A quad
                                takes one thread per Philox block of the
                                largest colour (a power of two up to 64);
                                the workgroup, rounded up to whole 64-lane
                                waves, has at most 1024 threads, and quads
                                of at most 64 threads must fill its waves  */
    int autotune;            /* 1: when tile_rows and group_replicas are 0,
                                pick them by timing the candidate shapes on
                                a throw-away run first (see pamc_autotune);
                                0 (default): a fixed rule                   */
    const int64_t *pop_schedule; /* NULL: the nominal population is R at every
                                step.  Else [n_temps] nominal populations
                                R(beta_k) (Sec. III.D), pop_schedule[0] = R,
                                all >= 1: the resampling to beta_{k+1}
                                targets pop_schedule[k+1], and the default
                                capacity follows the largest entry.  Read
                                during pamc_create only.                     */
    int real_couplings;      /* pamc_footprint and pamc_autotune only (they
                                take no couplings): 1 = size or tune a run
                                with real couplings                         */
    int icm_rounds;          /* isoenergetic cluster moves (Sec. IV): 0
                                (default) = none; n in [1, 8] = at every step
                                after a resampling, floor(sweeps/2) sweeps,
                                then n rounds that update floor(R_k/2)
                                disjoint random replica pairs each (the
                                paper's R updates per step: n = 2), then the
                                remaining sweeps.  An update flips, in both
                                replicas, the island of the smaller overlap
                                sector that holds a randomly drawn site.
                                Needs PAMC_SPINS_INT8.  Family ids stay with
                                their rows, so S_f and rho_s no longer
                                measure equilibration (use rho_f)          */
    double icm_beta_min;     /* cluster moves only at steps with beta_k >=
                                icm_beta_min (the paper restricts them to a
                                low-temperature window in 3D); 0 = every
                                step after a resampling                     */
    int dim;                 /* lattice dimension D (Sec. II.A studies both):
                                3 (default; 0 also means 3), or 2 = the
                                periodic L x L square lattice, site
                                s = x + L y, four neighbours, couplings
                                [2][L^2] (d = 0, 1 for x, y).  D = 2 takes
                                real couplings (pamc_create_real or
                                pamc_instance.real_couplings; +-J instances
                                as j = +-2^20) and 2 <= L <= 64.  Read by
                                pamc_footprint and pamc_autotune too.  The
                                serving API (pamc_server_*) is 3D only.     */
} pamc_options;

/* Fills *opt with the defaults described above. */
void pamc_default_options(pamc_options *opt);

/* Sweep workgroup shape for lattice size L, population R and `sweeps`
 * sweeps per step, chosen by measurement: after eight burn-in steps, each
 * candidate shape runs four temperature steps (one warm-up) of a
 * throw-away run with seeded +-J couplings at beta = 2, timed by HIP events
 * on opt's stream and device, and the shape with the fastest timed step
 * wins.  Results of a run never depend on the shape.
 * Choices are cached per process by (kernel, L, sweeps, capacity rounded up
 * to a power of two, opt's spin format); a cached shape is returned without
 * measuring.  The
 * throw-away run needs the device memory of one run of this size.
 * Outputs (each may be NULL): *tile_rows, *group_replicas (0 where the
 * kernel has a fixed value), *ns_per_attempt (sweep time per spin-flip
 * attempt of the winner).
 * Errors: PAMC_ERR_INVALID, PAMC_ERR_NOMEM, PAMC_ERR_DEVICE. */
int pamc_autotune(int L, int64_t R, int sweeps, const pamc_options *opt, int *tile_rows, int *group_replicas,
                  double *ns_per_attempt);

typedef struct pamc_ctx pamc_ctx;

/* Creates a run and initialises R random replicas at step 0 (Sec. II.B).
 *   L          linear size, 2 <= L <= 32 (N = L^3);
 *   couplings  int8 [3][N], +-1; couplings[d*N + s] joins site s and its
 *              periodic neighbour s + e_d (d = 0, 1, 2 for x, y, z; site
 *              s = x + L (y + L z));
 *   R          nominal population, 1 <= R; capacity must stay below 2^31;
 *   beta       double [n_temps], finite, non-decreasing, beta[0] = 0
 *              exactly: the replicas start as independent random spins,
 *              which is the beta = 0 equilibrium (Sec. II.B), and the free
 *              energy is anchored there at ln Z_0 = N ln 2 (any other
 *              beta[0] is PAMC_ERR_INVALID);
 *   sweeps     Metropolis sweeps per temperature, >= 1;
 *   seed       Philox key;
 *   opt        NULL for defaults.
 * Errors: PAMC_ERR_INVALID, PAMC_ERR_NOMEM, PAMC_ERR_DEVICE. */
int pamc_create(int L, const int8_t *couplings, int64_t R, const double *beta, int n_temps,
                int sweeps, uint64_t seed, const pamc_options *opt, pamc_ctx **out);

/* The same with real couplings (Sec. II.A: the paper's case study draws them
 * from a Gaussian of mean 0 and variance 1), in fixed point:
 *   couplings  int32 [D][N], J = couplings[d*N + s] * 2^-20 with
 *              |couplings| < 2^23 (|J| < 8), same bond order as pamc_create
 *              (D = opt->dim: [3][L^3], or [2][L^2] on the square lattice);
 *   L          3D: even L <= 20 or odd L <= 21 (the colour-major sweep);
 *              2D: 2 <= L <= 64;
 *   capacity   at most 2^29, and times the sum of |couplings| below 2^62.
 * Energies are exact integers in units of 2^-20 (the E_min, E_max, sum_E,
 * sum_E2 fields of pamc_step_obs and pamc_state.E_fixed); mean_E, e, C_V,
 * lnQ and the free energies are in energy units.  Metropolis acceptance of
 * a move with dE > 0: u < floor(e 2^32) with e = exp(-beta dE) evaluated by
 * a fixed binary32 recipe (Cody-Waite reduction, degree-7 Taylor polynomial
 * with fused multiply-adds); resampling weights per replica as the product
 * over the set bits b of E - E_min of exp(-dbeta 2^(b-20)).  Errors as for
 * pamc_create. */
int pamc_create_real(int L, const int32_t *couplings, int64_t R, const double *beta, int n_temps,
                     int sweeps, uint64_t seed, const pamc_options *opt, pamc_ctx **out);

/* Runs up to n_steps temperature steps (n_steps < 0: to the end); a step k
 * is the sweeps at beta_k, the measurements, and for k < n_temps - 1 the
 * resampling to beta_{k+1}.  Returns PAMC_OK when the requested steps (or
 * the run) finished.  PAMC_ERR_CAPACITY / PAMC_ERR_EXTINCT: the step whose
 * resampling failed is not applied; the handle keeps the population of that
 * step after its sweeps, and the failure is sticky.  Synchronises the
 * stream before returning. */
int pamc_anneal(pamc_ctx *ctx, int n_steps);

/* Enqueues up to n_steps steps without waiting; the result is read by
 * pamc_sync.  For timing and overlap with other host work. */
int pamc_anneal_async(pamc_ctx *ctx, int n_steps);
int pamc_sync(pamc_ctx *ctx);

/* Per-step observables, measured after the sweeps at beta_k. */
typedef struct pamc_step_obs {
    double beta;
    int64_t R;          /* population R_k                                  */
    int64_t sum_E;      /* sum of energies (exact; units of 2^-20 for real
                           couplings)                                      */
    int64_t sum_E2;     /* sum of squared energies (exact): low 64 bits    */
    int64_t sum_E2_hi;  /*   and high 64 bits (0 for +-1 couplings)        */
    int64_t E_min, E_max;
    double mean_E;      /* sum_E / R_k                                     */
    double e;           /* mean_E / N                                      */
    double C_V;         /* beta^2 var(E) / N, var from the exact sums      */
    double lnQ;         /* ln[(1/R_k) sum_i exp(-(beta_{k+1}-beta_k) E_i)]; NaN at the last step */
    double lnZ;         /* N ln 2 + sum_{j<k} lnQ_j                       */
    double betaF;       /* -lnZ                                           */
    double f;           /* -lnZ / (beta N); NaN at beta = 0               */
    double S_f;         /* family entropy, Eq. (2)                        */
    double rho_s;       /* R_k / exp(S_f)                                 */
    double q_abs, q2, q4, g_SG; /* overlap moments and Binder cumulant at
                                   overlap steps, NaN elsewhere            */
    int32_t measured;   /* 1 once step k has run                           */
} pamc_step_obs;

/* Copies the observables of steps 0 .. n-1 (n <= n_temps) into out[n]. */
int pamc_observables(const pamc_ctx *ctx, pamc_step_obs *out, int n);

/* Overlap histogram of step k: hist[Q + N] for Q = sum_s S^a_s S^b_s over
 * the pairs (r, r + floor(R_k/2)), r < floor(R_k/2); int64 [2N+1].
 * PAMC_ERR_STATE if k is not an overlap step or has not run. */
int pamc_overlap_hist(const pamc_ctx *ctx, int step, int64_t *hist);

/* Per-step normalisers: S_k = sum over the population of
 * exp(-(beta_{k+1}-beta_k)(E_i - E_min)) as summed by the library, and the
 * family term T_k = sum_i n_i ln n_i.  double [n] each; NULL to skip. */
int pamc_step_sums(const pamc_ctx *ctx, double *S, double *T, int n);

/* Population state.  spins: int8 [R_k][N] of +-1 in lexicographic site
 * order; E: int32 [R_k] (+-1 couplings); family: uint32 [R_k] (index of the
 * initial replica each row descends from, non-decreasing); E_fixed: int64
 * [R_k] energies in units of 2^-20 (real couplings). */
typedef struct pamc_state {
    int step;        /* next step to run, 0 .. n_temps                    */
    int64_t R;       /* R_k                                               */
    double lnZ;      /* ln Z_k                                            */
    int8_t *spins;
    int32_t *E;      /* +-1 couplings only; untouched for real couplings  */
    uint32_t *family;
    int64_t *E_fixed;/* real couplings only; untouched for +-1 couplings  */
} pamc_state;

/* Reads the current step and population size (no copies). */
int pamc_get_shape(const pamc_ctx *ctx, int *step, int64_t *R);
/* Sweep workgroup shape the run uses (see tile_rows, group_replicas). */
int pamc_sweep_shape(const pamc_ctx *ctx, int *tile_rows, int *group_replicas);

/* Copies the current population into the caller's buffers (sized by
 * pamc_get_shape); any NULL array is skipped. */
int pamc_get_state(pamc_ctx *ctx, pamc_state *st);

/* Replaces the population (checkpoint resume, step-wise checks): step in
 * [0, n_temps), 1 <= R <= capacity, spins +-1, family < R (nominal).
 * Energies are recomputed from the spins; st->E is ignored. */
int pamc_set_state(pamc_ctx *ctx, const pamc_state *st);

/* Metropolis thresholds of every step: out[k][0..2] for dE = 4, 8, 12,
 * accept_all[k] = 1 when beta_k = 0 (every move accepted).  PAMC_ERR_STATE
 * for real couplings (their acceptance is evaluated per move). */
int pamc_thresholds(const pamc_ctx *ctx, uint32_t *out, uint8_t *accept_all);

/* Device time of the steps run since the previous call (options.timing =
 * 1), measured with HIP events on the run's stream:
 *   sweep_ms     the sweep kernels (sweeps of all replicas, energies,
 *                energy histogram, measurement and the resampling table);
 *   resample_ms  copy counts, family and overlap statistics, prefix sum and
 *                copy map;
 *   gather_ms    the stand-alone gather of surviving replicas (zero when the
 *                gather is fused into the next sweep, fuse_gather = 1);
 *   n_steps      the number of steps.
 * Any output may be NULL.  PAMC_ERR_STATE if timing is off. */
int pamc_phase_times(pamc_ctx *ctx, double *sweep_ms, double *resample_ms, double *gather_ms,
                     int64_t *n_steps);

/* +-J instance generator (Sec. II.A: couplings +-1 with probability 1/2
 * each; the paper's instances are not published).  Fills out, int8
 * [3][L^3] in the bond order of pamc_create, with out[b] for bond
 * b = d L^3 + s equal to +1 when bit 31 of word (b & 3) of Philox4x32-10
 * at counter (b >> 2, 0, 0, 5 * 2^28), key (low, high 32 bits of
 * disorder_seed), is set, else -1.  Host only (no device, no allocation);
 * 2 <= L <= 32; out has 3 L^3 bytes, caller-owned.
 * Errors: PAMC_ERR_INVALID. */
int pamc_make_pm_j(int L, uint64_t disorder_seed, int8_t *out);

/* Free-energy variance of Eq. (4) (Sec. II.B), rho_f = R var(beta F), over
 * independent runs of one instance at finite R:
 *   betaF       double [runs][n_temps], beta F_k of each run (host);
 *   nominal_R   double [n_temps], the nominal population R(beta_k);
 *   outputs     double [n_temps] each, NULL to skip: the mean of beta F,
 *               its sample variance (ddof 1: the sum of squared deviations
 *               from the mean over runs - 1), and rho_f = R(beta_k) times
 *               that variance.
 * Sums run over the runs in order, in FP64.  runs >= 2.  Host only.
 * Errors: PAMC_ERR_INVALID. */
int pamc_rho_f(const double *betaF, int runs, int n_temps, const double *nominal_R, double *mean_betaF,
               double *var_betaF, double *rho_f);

/* Calibration of the sweep's roofline on a device (-1 = current): the
 * rate of a kernel that only draws Philox4x32-10 blocks with the sweep's
 * counter pattern (counter (block, replica, step, TAG_SWEEP | sweep), ten
 * sweeps per replica, the four words XOR-folded), in 32-bit words per ns,
 * and the rate of a kernel of independent three-input XORs and adds, in
 * int32 VALU operations per ns.  The sweep draws one word per attempted
 * flip (Sec. III.A), so the first rate bounds its attempts per ns.  Each
 * output may be NULL.  Allocates and frees a small device buffer.
 * Errors: PAMC_ERR_NOMEM, PAMC_ERR_DEVICE. */
int pamc_calibrate(int device, double *philox_words_per_ns, double *valu_ops_per_ns);

/* Device footprint in bytes of a run with these parameters; -1 for
 * arguments no run accepts. */
int64_t pamc_footprint(int L, int64_t R, int n_temps, const pamc_options *opt);

void pamc_destroy(pamc_ctx *ctx);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run
 * of pamc_create + pamc_anneal + pamc_observables (+ pamc_get_state) with
 * default options and +-1 couplings, in one call that allocates no device
 * memory.  Every device buffer comes from one array of 64 MiB that the
 * library holds on each GPU it runs on until the process ends; runs that
 * need more (about 2 capacity rows of L^3 bytes plus tables) are refused
 * with PAMC_ERR_INVALID before any device work.  Arguments as in
 * pamc_create; stream: the hipStream_t to run on (NULL: the null stream);
 * the call returns after the run has finished.
 *   obs          pamc_step_obs [n_temps], caller-owned, filled as by
 *                pamc_observables;
 *   final_state  NULL, or caller buffers as in pamc_get_state sized for the
 *                capacity R + ceil(8 sqrt R) + 64 rows; st->R gives the rows
 *                written.
 * Results equal those of pamc_create + pamc_anneal for the same arguments.
 * All calls on one GPU share its array, which keeps the last call's
 * contents (each call clears what must start at zero): calls from one
 * process are serialised by a lock; calls whose device work overlapped
 * would race.  Returns PAMC_OK, PAMC_ERR_CAPACITY or PAMC_ERR_EXTINCT (the
 * observables up to the failing step are still filled), PAMC_ERR_INVALID,
 * PAMC_ERR_NOMEM (the estimate of the array's use fell short) or
 * PAMC_ERR_DEVICE. */
int pamc_anneal_static(int L, const int8_t *couplings, int64_t R, const double *beta, int n_temps, int sweeps,
                       uint64_t seed, void *stream, pamc_step_obs *obs, pamc_state *final_state);

const char *pamc_status_string(int status);
const char *pamc_last_error(void);

/* ------------------------------------------------------------------------ */
/* Batched form: many independent instances of mixed L annealed together.   */
/* Results equal those of separate pamc_create/pamc_anneal runs.            */
/* ------------------------------------------------------------------------ */
typedef struct pamc_instance {
    int L;
    const int8_t *couplings; /* [3][L^3] */
    int64_t R;
    const double *beta;      /* [n_temps] */
    int n_temps;
    int sweeps;
    uint64_t seed;
    const int64_t *pop_schedule; /* NULL or [n_temps], as in pamc_options */
    const int32_t *real_couplings; /* NULL: couplings (+-1) above; else
                                 [D][L^D] real couplings as in
                                 pamc_create_real (couplings is ignored);
                                 D is the batch options' dim            */
} pamc_instance;

typedef struct pamc_batch pamc_batch;

/* With opt->autotune and no explicit shape, the instances of one lattice
 * size (and kernel) share the shape tuned for their summed population, up to
 * 2e5 rows: they sweep as one launch per step. */
int pamc_batch_create(int n, const pamc_instance *inst, const pamc_options *opt, pamc_batch **out);
int pamc_batch_anneal(pamc_batch *b);
int pamc_batch_observables(const pamc_batch *b, int i, pamc_step_obs *out, int n);
int pamc_batch_get_state(pamc_batch *b, int i, pamc_state *st);
int pamc_batch_shape(const pamc_batch *b, int i, int *step, int64_t *R);
void pamc_batch_destroy(pamc_batch *b);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop that admits instances while others run.          */
/* ------------------------------------------------------------------------ */
typedef struct pamc_server pamc_server;

typedef struct pamc_server_options {
    int max_active;      /* most instances on the device at once (0 = 256) */
    int device;          /* -1 = current                                    */
    int autotune;        /* 1: each request's sweep shape is chosen by
                            measurement at submission (pamc_autotune, cached
                            per process and in the shipped tuning file),
                            for a population of 10^5 rows of the request's
                            lattice: requests of one size sweep together in
                            one launch, whatever their own R; 0: the fixed
                            rule                                            */
    int spin_format;     /* PAMC_SPINS_INT8 or PAMC_SPINS_PACKED for every
                            request (footprints follow it)                  */
} pamc_server_options;

typedef struct pamc_result {
    int status;                /* PAMC_OK or the error of this request     */
    int n_temps;
    pamc_step_obs *obs;        /* caller buffer [n_temps], filled on success */
    double submit_time_s;      /* host clock, seconds                      */
    double admit_time_s;
    double finish_time_s;
} pamc_result;

/* hbm_budget_bytes bounds the device memory of admitted requests: a
 * request holds pamc_footprint(L, R, n_temps, options with the server's
 * spin format) + 4096 bytes of it from admission to completion. */
int pamc_server_create(size_t hbm_budget_bytes, const pamc_server_options *opt, pamc_server **out);
/* Thread-safe.  PAMC_ERR_REJECTED if the request alone exceeds the budget. */
int pamc_server_submit(pamc_server *s, const pamc_instance *inst, uint64_t *req_id);
/* PAMC_ERR_BUSY while the request is queued or running. */
int pamc_server_poll(pamc_server *s, uint64_t req_id, pamc_result *out);
int pamc_server_cancel(pamc_server *s, uint64_t req_id);
/* Counters: completed, queued, active. */
int pamc_server_stats(pamc_server *s, int64_t *completed, int64_t *queued, int64_t *active);
/* Memory and device use (each output may be NULL): used_bytes, the budget
 * held by admitted requests (0 when none runs); budget_bytes, the budget;
 * busy_s, the device time spent running temperature steps since creation
 * (HIP events around every batch of steps); wall_s, the host time since
 * creation.  Returns the loop's status. */
int pamc_server_usage(pamc_server *s, size_t *used_bytes, size_t *budget_bytes, double *busy_s, double *wall_s);
void pamc_server_destroy(pamc_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PAMC_H */
