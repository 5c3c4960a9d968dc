/* Drives the oracle through every mode on small instances, so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer checks its memory
 * accesses and arithmetic: +-J and real couplings, the square lattice,
 * isoenergetic cluster moves, a population schedule, overlap steps, a
 * capacity failure, set_state / measure_resample / sweep_rows, the
 * observables and the exact enumeration.  Exits non-zero on a failed
 * check; the sanitizers abort on their own findings. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc orc_t;
orc_t *orc_create(int L, const int8_t *J, int64_t R, int64_t Rcap, const double *beta, int nT, int NS, uint64_t seed,
                  const uint8_t *overlap_steps, const int64_t *pop);
orc_t *orc_create_real_dim(int dim, int L, const int32_t *Jq, int64_t R, int64_t Rcap, const double *beta, int nT,
                           int NS, uint64_t seed, const uint8_t *overlap_steps, const int64_t *pop);
void orc_destroy(orc_t *o);
void orc_set_threads(orc_t *o, int n);
void orc_set_icm(orc_t *o, int rounds, double beta_min);
int orc_run(orc_t *o, int n_steps);
int64_t orc_population(const orc_t *o);
int orc_get_state(const orc_t *o, int8_t *spins, int32_t *E, uint32_t *fam);
int orc_set_state(orc_t *o, int k, int64_t Rk, const int8_t *spins, const uint32_t *fam, double lnZ);
int orc_sweep_rows(orc_t *o, int k, int64_t n, const int64_t *rows, int8_t *spins, int32_t *E);
int orc_measure_resample(orc_t *o);
int orc_records(const orc_t *o, int64_t *ints, double *dbl, int64_t *qhist);
int orc_observables(const orc_t *o, double *out, double *ovl_out);
int orc_make_pm_j(int L, uint64_t seed, int8_t *out);
int enum_dos(int L, const int8_t *J, int64_t *g);

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

static double *linear_beta(int nT, double bmax)
{
    double *b = malloc(sizeof(double) * nT);
    for (int k = 0; k < nT; ++k) b[k] = nT > 1 ? bmax * k / (nT - 1) : 0.0;
    return b;
}

static int run_pm(int L, int64_t R, int nT, int NS, int icm, int threads)
{
    const int N = L * L * L;
    int8_t *J = malloc(3 * N);
    CHECK(orc_make_pm_j(L, 77 + L, J) == 0);
    double *beta = linear_beta(nT, 4.0);
    uint8_t *ovl = calloc(nT, 1);
    ovl[nT / 2] = ovl[nT - 1] = 1;
    int64_t *pop = malloc(sizeof(int64_t) * nT);
    for (int k = 0; k < nT; ++k) pop[k] = k == 0 ? R : R - k;
    const int64_t cap = R + 64 + 8 * 40;
    orc_t *o = orc_create(L, J, R, cap, beta, nT, NS, 5 + L, ovl, pop);
    CHECK(o != NULL);
    orc_set_threads(o, threads);
    if (icm) orc_set_icm(o, icm, 0.5);
    CHECK(orc_run(o, nT / 2) == 0);
    const int64_t Rk = orc_population(o);
    int8_t *sp = malloc((size_t)cap * N);
    int32_t *E = malloc(sizeof(int32_t) * cap);
    uint32_t *f = malloc(sizeof(uint32_t) * cap);
    CHECK(orc_get_state(o, sp, E, f) == 0);
    int64_t rows[3] = {0, Rk / 2, Rk - 1};
    int8_t *s3 = malloc(3 * (size_t)N);
    for (int i = 0; i < 3; ++i) memcpy(s3 + (size_t)i * N, sp + (size_t)rows[i] * N, N);
    int32_t E3[3];
    CHECK(orc_sweep_rows(o, nT / 2, 3, rows, s3, E3) == 0);
    CHECK(orc_run(o, -1) == 0);
    int64_t *ints = malloc(sizeof(int64_t) * 8 * nT);
    double *dbl = malloc(sizeof(double) * 8 * nT);
    int64_t *q = malloc(sizeof(int64_t) * nT * (2 * N + 1));
    CHECK(orc_records(o, ints, dbl, q) == 0);
    double *obs = malloc(sizeof(double) * 16 * nT);
    double *ov = malloc(sizeof(double) * 8 * nT);
    CHECK(orc_observables(o, obs, ov) == 0);
    /* resume from the mid-run state and measure / resample without sweeps */
    orc_t *p = orc_create(L, J, R, cap, beta, nT, NS, 5 + L, NULL, pop);
    CHECK(p != NULL);
    CHECK(orc_set_state(p, nT / 2, Rk, sp, f, 1.0) == 0);
    CHECK(orc_measure_resample(p) == 0);
    orc_destroy(p);
    orc_destroy(o);
    /* a capacity too small fails cleanly */
    o = orc_create(L, J, R, R, beta, nT, NS, 9, NULL, NULL);
    CHECK(o != NULL);
    const int st = orc_run(o, -1);
    CHECK(st == 0 || st == -3);
    orc_destroy(o);
    free(J); free(beta); free(ovl); free(pop); free(sp); free(E); free(f); free(s3);
    free(ints); free(dbl); free(q); free(obs); free(ov);
    return 0;
}

static int run_real(int dim, int L, int64_t R, int nT, int icm)
{
    const int N = dim == 3 ? L * L * L : L * L;
    int32_t *Jq = malloc(sizeof(int32_t) * dim * N);
    uint32_t x = 12345u + (uint32_t)L;
    for (int i = 0; i < dim * N; ++i) {
        x = x * 1664525u + 1013904223u;
        Jq[i] = (int32_t)(x >> 9) - (1 << 22);
    }
    double *beta = linear_beta(nT, 3.0);
    orc_t *o = orc_create_real_dim(dim, L, Jq, R, R + 400, beta, nT, 4, 3, NULL, NULL);
    CHECK(o != NULL);
    if (icm) orc_set_icm(o, icm, 0.0);
    CHECK(orc_run(o, -1) == 0);
    double *obs = malloc(sizeof(double) * 16 * nT);
    double *ov = malloc(sizeof(double) * 8 * nT);
    CHECK(orc_observables(o, obs, ov) == 0);
    orc_destroy(o);
    free(Jq); free(beta); free(obs); free(ov);
    return 0;
}

int main(void)
{
    for (int L = 2; L <= 7; ++L) CHECK(run_pm(L, 300, 9, 3, 0, 1) == 0);
    CHECK(run_pm(8, 400, 7, 2, 2, 4) == 0);
    CHECK(run_pm(5, 200, 7, 2, 2, 2) == 0);
    CHECK(run_real(3, 4, 200, 7, 0) == 0);
    CHECK(run_real(3, 5, 150, 7, 2) == 0);
    CHECK(run_real(2, 9, 300, 7, 2) == 0);
    CHECK(run_real(2, 8, 300, 7, 2) == 0);
    int8_t J[3 * 8];
    CHECK(orc_make_pm_j(2, 1, J) == 0);
    int64_t g[3 * 8 + 1];
    CHECK(enum_dos(2, J, g) == 0);
    int64_t tot = 0;
    for (int m = 0; m <= 3 * 8; ++m) tot += g[m];
    CHECK(tot == 256);
    printf("oracle sanitizer run ok\n");
    return 0;
}
