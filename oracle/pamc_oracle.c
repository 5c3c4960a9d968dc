/*
 * pamc_oracle.c -- plain CPU population annealing Monte Carlo (PAMC) for the
 * Edwards-Anderson Ising spin glass on the periodic cubic (D = 3) lattice, and
 * with real couplings also on the periodic square (D = 2) lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct oracle that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Couplings are either +-1 or real, the paper's own case study (Sec. II.A:
 * Gaussian, mean 0, variance 1), held in fixed point as J = j 2^-20 with an
 * integer j, |J| < 8, so that energies are exact integers in units of 2^-20
 * and every sum is independent of its order.
 *
 * Paper: A. Barzegar, C. Pattison, W. Wang, H. G. Katzgraber, "Optimization
 * of population annealing Monte Carlo for large-scale spin-glass simulations"
 * (arXiv:1710.09025).  Passages followed:
 *   Sec. II.A, Eq. (1)   H = -sum_<ij> J_ij S_i S_j, nearest neighbours on an
 *                        L^D lattice, N = L^D spins.
 *   Sec. II.B            PAMC outline: R replicas initialised at random at
 *                        beta = 0; on each lowering beta -> beta' the mean
 *                        number of copies of replica i is proportional to
 *                        exp[-(beta'-beta) E_i], normalised so that the
 *                        expected new population is R(beta'); then N_S
 *                        Metropolis sweeps per replica, one sweep being N
 *                        attempted spin updates.
 *   Sec. II.B, Eq. (2)   family entropy S_f = -sum_i nu_i ln nu_i and the
 *                        entropic family size rho_s = R / e^{S_f}; the free
 *                        energy by free-energy perturbation.
 *   Sec. III.A           checkerboard spin selection on bipartite lattices.
 *   Sec. III.D           rho_s uses the local population size R at each beta.
 *   Sec. IV (Houdayer)   isoenergetic cluster moves (ICM): after a
 *                        resampling, N_S/2 sweeps, then R updates of random
 *                        replica pairs, then N_S/2 sweeps; an update builds
 *                        the overlap of the pair, takes an island of the
 *                        sector with fewer sites and flips it in both
 *                        replicas (their summed energy is unchanged).
 *   Sec. V.A, Eq. (9)    observables are population averages; the spin
 *                        overlap is measured only at selected temperatures.
 *
 * Readings where the paper is silent (the design notes list every one):
 *   periodic boundaries; +-J couplings; for odd L a three-colouring
 *   c = (g(x)+g(y)+g(z)) mod 3 with g(v) = v mod 2 for v < L-1 and
 *   g(L-1) = 2 (in 2D the same with z = 0, g(0) = 0); 2D only with real
 *   couplings (+-J instances enter as real couplings of magnitude 1); a Philox4x32-10 counter contract for every random number;
 *   Metropolis acceptance as a uint32 threshold compare; nearest-integer
 *   (floor/ceil) resampling normalised to the nominal R; weights taken
 *   relative to E_min as a fixed product of powers of exp(-2 dbeta); a
 *   pairwise summation tree for the normaliser and for the family term;
 *   the order sweep -> measure -> resample at every beta_k, beta_0 included.
 * For real couplings: the fixed-point couplings above; Metropolis acceptance
 *   u < floor(e 2^32) with e = exp(-beta dE) evaluated in binary32 by the
 *   function orc_exp_f32 below; per-replica weights relative to E_min as a
 *   fixed product of exp(-dbeta 2^(b-20)) over the set bits b of E - E_min;
 *   the normaliser summed by the pairwise tree over replica rows.
 * For ICM: the R updates as two rounds of floor(R_k/2) disjoint pairs, rows
 *   paired by a keyed pseudo-random permutation (a four-round Feistel
 *   network on 2h-bit words whose round function is Philox, cycle-walked
 *   into [0, R_k)); the island is the one containing a uniformly drawn site
 *   of the smaller sector (ties: the sector where the replicas differ; an
 *   empty sector is no move); ICM at every step k >= 1 (optionally only
 *   where beta_k >= a given minimum, the low-temperature window in which
 *   the paper finds the moves efficient in 3D), after floor(N_S/2) sweeps;
 *   family ids stay with their rows.
 *
 * Spins are stored as int8 +-1, replica-major, sites in lexicographic order
 * s = x + L (y + L z).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORC_OK = 0,
    ORC_ERR_INVALID = -1,
    ORC_ERR_NOMEM = -2,
    ORC_ERR_CAPACITY = -3,
    ORC_ERR_EXTINCT = -4,
    ORC_ERR_STATE = -6
};

/* Philox stream tags, the top four bits of counter word 3. */
#define TAG_INIT 0x10000000u
#define TAG_SWEEP 0x20000000u
#define TAG_RESAMPLE 0x30000000u
#define TAG_ICM 0x40000000u
#define TAG_COUPLING 0x50000000u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications    */
/* with the round key added by XOR, the key bumped by the Weyl constants     */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static uint32_t draw(uint64_t seed, uint32_t x, uint32_t y, uint32_t z, uint32_t w, int word)
{
    uint32_t ctr[4] = {x, y, z, w};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word];
}

/* +-J disorder (Sec. II.A: each coupling +1 or -1 with probability 1/2;
 * the instances of the paper are not published).  Bond b = d N + s of the
 * [3][N] array is +1 when bit 31 of word (b & 3) of the Philox block at
 * counter (b >> 2, 0, 0, TAG_COUPLING), keyed by the disorder seed, is set. */
int orc_make_pm_j(int L, uint64_t disorder_seed, int8_t *out)
{
    if (L < 2 || L > 32 || !out) return ORC_ERR_INVALID;
    const int64_t nb = 3 * (int64_t)L * L * L;
    for (int64_t b = 0; b < nb; ++b) {
        uint32_t u = draw(disorder_seed, (uint32_t)(b >> 2), 0u, 0u, TAG_COUPLING, (int)(b & 3));
        out[b] = (u >> 31) ? 1 : -1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* State                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim, L, N, ncol;  /* N = L^dim; 2 dim neighbours per site         */
    int64_t R, Rcap;
    int nT, NS;
    uint64_t seed;
    double *beta;
    int64_t *Rt;          /* [nT] nominal population at each beta_k, Rt[0] = R */
    int gauss;      /* 1: real couplings in fixed point (units of 2^-20)  */
    int8_t *J;      /* [dim][N]: bond (s, d) joins s and s + e_d (+-1)    */
    int32_t *Jq;    /* [dim][N]: the same for real couplings, J = Jq 2^-20 */
    int *nbr;       /* [N][6]: +x, -x, +y, -y, +z, -z (the first 2 dim)   */
    int8_t *Jn;     /* [N][6]: coupling of the bond to that neighbour     */
    int32_t *Jnq;   /* [N][6]: the same for real couplings                */
    int *colour;    /* [N]                                                */
    int *crank;     /* [N]: rank of s among sites of its colour           */
    int8_t *spin, *spin2;
    int64_t *E, *E2; /* energies (units of 2^-20 for real couplings)       */
    uint32_t *fam, *fam2;
    uint32_t *ncopy;
    int64_t Rk;
    int k;
    double lnZ;
    uint8_t *ovl;   /* [nT]: measure the overlap at this step             */
    int nthreads;
    int icm_rounds;  /* ICM rounds of disjoint pairs per step (0: none)   */
    double icm_beta_min; /* ICM only at steps with beta_k >= this        */
    /* per-step records */
    int64_t *o_R, *o_sumE;
    __int128 *o_sumE2;
    int64_t *o_Emin, *o_Emax;
    double *o_S, *o_T, *o_lnQ, *o_lnZ;
    int64_t *o_q; /* [nT][2N+1] */
} orc_t;

static int site(int L, int x, int y, int z) { return x + L * (y + L * z); }

/* Colour of a site (Sec. III.A checkerboard; three colours for odd L). */
static int colour_of(int L, int x, int y, int z)
{
    if (L % 2 == 0) return (x + y + z) % 2;
    int gx = (x == L - 1) ? 2 : x % 2;
    int gy = (y == L - 1) ? 2 : y % 2;
    int gz = (z == L - 1) ? 2 : z % 2;
    return (gx + gy + gz) % 3;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    free(o->beta);
    free(o->Rt);
    free(o->J);
    free(o->Jq);
    free(o->nbr);
    free(o->Jn);
    free(o->Jnq);
    free(o->colour);
    free(o->crank);
    free(o->spin);
    free(o->spin2);
    free(o->E);
    free(o->E2);
    free(o->fam);
    free(o->fam2);
    free(o->ncopy);
    free(o->ovl);
    free(o->o_R);
    free(o->o_sumE);
    free(o->o_sumE2);
    free(o->o_Emin);
    free(o->o_Emax);
    free(o->o_S);
    free(o->o_T);
    free(o->o_lnQ);
    free(o->o_lnZ);
    free(o->o_q);
    free(o);
}

/* Coupling of bond (s, d), in units of 2^-20 for real couplings. */
static int64_t coupling(const orc_t *o, int d, int s)
{
    return o->gauss ? (int64_t)o->Jq[d * o->N + s] : (int64_t)o->J[d * o->N + s];
}

/* Energy of one replica, Eq. (1): each of the dim N bonds counted once. */
static int64_t energy(const orc_t *o, const int8_t *S)
{
    int64_t e = 0;
    for (int s = 0; s < o->N; ++s)
        for (int d = 0; d < o->dim; ++d) e -= coupling(o, d, s) * S[s] * S[o->nbr[s * 6 + 2 * d]];
    return e;
}

/* Random initial replicas at beta = 0 (Sec. II.B): S = +1 when bit 31 of the
 * INIT draw is set. */
static void init_population(orc_t *o)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t r = 0; r < o->R; ++r) {
        int8_t *S = o->spin + r * o->N;
        for (int s = 0; s < o->N; ++s) {
            uint32_t u = draw(o->seed, (uint32_t)(s >> 2), (uint32_t)r, 0u, TAG_INIT, s & 3);
            S[s] = (u >> 31) ? 1 : -1;
        }
        o->E[r] = energy(o, S);
        o->fam[r] = (uint32_t)r;
    }
    o->Rk = o->R;
    o->k = 0;
    o->lnZ = (double)o->N * log(2.0);
}

/* pop: NULL for a constant nominal population R, or the nominal population
 * R(beta_k) of every step (pop[0] = R), Sec. III.D. */
static orc_t *create(int dim, int L, const int8_t *J, const int32_t *Jq, int64_t R, int64_t Rcap,
                     const double *beta, int nT, int NS, uint64_t seed, const uint8_t *overlap_steps,
                     const int64_t *pop)
{
    if (dim != 2 && dim != 3) return NULL;
    if (dim == 2 && !Jq) return NULL;
    if (L < 2 || L > (dim == 3 ? 32 : 64) || R < 1 || nT < 1 || NS < 1 || (!J && !Jq) || !beta) return NULL;
    if (Rcap < R) return NULL;
    if (pop) {
        if (pop[0] != R) return NULL;
        for (int i = 0; i < nT; ++i)
            if (pop[i] < 1) return NULL;
    }
    /* Sec. II.B: the replicas start at random, the beta = 0 sample, which is
     * also where ln Z = N ln 2 anchors the free energy */
    if (beta[0] != 0.0) return NULL;
    for (int i = 0; i < nT; ++i) {
        if (!(beta[i] >= 0.0) || !isfinite(beta[i])) return NULL;
        if (i > 0 && beta[i] < beta[i - 1]) return NULL;
    }
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    if (!o) return NULL;
    o->dim = dim;
    o->L = L;
    o->N = dim == 3 ? L * L * L : L * L;
    o->gauss = Jq != NULL;
    o->ncol = (L % 2 == 0) ? 2 : 3;
    o->R = R;
    o->Rcap = Rcap;
    o->nT = nT;
    o->NS = NS;
    o->seed = seed;
    o->nthreads = 1;
    int N = o->N;
    o->beta = (double *)malloc(sizeof(double) * nT);
    o->Rt = (int64_t *)malloc(sizeof(int64_t) * nT);
    if (o->Rt)
        for (int i = 0; i < nT; ++i) o->Rt[i] = pop ? pop[i] : R;
    o->J = (int8_t *)calloc((size_t)dim * N, 1);
    o->Jq = (int32_t *)calloc((size_t)dim * N, sizeof(int32_t));
    o->nbr = (int *)malloc(sizeof(int) * 6 * (size_t)N);
    o->Jn = (int8_t *)calloc(6 * (size_t)N, 1);
    o->Jnq = (int32_t *)calloc(6 * (size_t)N, sizeof(int32_t));
    o->colour = (int *)malloc(sizeof(int) * N);
    o->crank = (int *)malloc(sizeof(int) * N);
    o->spin = (int8_t *)malloc((size_t)Rcap * N);
    o->spin2 = (int8_t *)malloc((size_t)Rcap * N);
    o->E = (int64_t *)malloc(sizeof(int64_t) * Rcap);
    o->E2 = (int64_t *)malloc(sizeof(int64_t) * Rcap);
    o->fam = (uint32_t *)malloc(sizeof(uint32_t) * Rcap);
    o->fam2 = (uint32_t *)malloc(sizeof(uint32_t) * Rcap);
    o->ncopy = (uint32_t *)malloc(sizeof(uint32_t) * Rcap);
    o->ovl = (uint8_t *)calloc(nT, 1);
    o->o_R = (int64_t *)calloc(nT, sizeof(int64_t));
    o->o_sumE = (int64_t *)calloc(nT, sizeof(int64_t));
    o->o_sumE2 = (__int128 *)calloc(nT, sizeof(__int128));
    o->o_Emin = (int64_t *)calloc(nT, sizeof(int64_t));
    o->o_Emax = (int64_t *)calloc(nT, sizeof(int64_t));
    o->o_S = (double *)calloc(nT, sizeof(double));
    o->o_T = (double *)calloc(nT, sizeof(double));
    o->o_lnQ = (double *)calloc(nT, sizeof(double));
    o->o_lnZ = (double *)calloc(nT, sizeof(double));
    o->o_q = (int64_t *)calloc((size_t)nT * (2 * N + 1), sizeof(int64_t));
    if (!o->beta || !o->Rt || !o->J || !o->Jq || !o->nbr || !o->Jn || !o->Jnq || !o->colour || !o->crank || !o->spin || !o->spin2 ||
        !o->E || !o->E2 || !o->fam || !o->fam2 || !o->ncopy || !o->ovl || !o->o_R || !o->o_sumE ||
        !o->o_sumE2 || !o->o_Emin || !o->o_Emax || !o->o_S || !o->o_T || !o->o_lnQ || !o->o_lnZ ||
        !o->o_q) {
        orc_destroy(o);
        return NULL;
    }
    memcpy(o->beta, beta, sizeof(double) * nT);
    if (J) {
        for (int i = 0; i < dim * N; ++i) {
            if (J[i] != 1 && J[i] != -1) {
                orc_destroy(o);
                return NULL;
            }
            o->J[i] = J[i];
        }
    } else {
        /* |J| < 8; the largest |E| (the sum of |j|) times the capacity stays
         * below 2^62, so sums of energies fit int64 and the variance numerator
         * R sum E^2 - (sum E)^2 fits int128 */
        int64_t A = 0;
        for (int i = 0; i < dim * N; ++i) {
            if (Jq[i] <= -(1 << 23) || Jq[i] >= (1 << 23)) {
                orc_destroy(o);
                return NULL;
            }
            o->Jq[i] = Jq[i];
            A += Jq[i] < 0 ? -(int64_t)Jq[i] : (int64_t)Jq[i];
        }
        if (A > 0 && (__int128)A * Rcap >= ((__int128)1 << 62)) {
            orc_destroy(o);
            return NULL;
        }
    }
    if (overlap_steps)
        memcpy(o->ovl, overlap_steps, nT);
    else
        o->ovl[nT - 1] = 1;

    /* Lattice (Sec. II.A): periodic neighbours and the coupling of each of
     * the 2 dim bonds of a site.  Bond (s, d) is stored at J[d][s] and joins
     * s to s + e_d, so the bond to s - e_d is J[d][s - e_d].  For L = 2 the
     * two x-neighbours coincide but the two bonds stay distinct.  In 2D the
     * z entries of the tables are never read. */
    int count[3] = {0, 0, 0};
    const int Lz = dim == 3 ? L : 1;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int s = site(L, x, y, z);
                int xp = site(L, (x + 1) % L, y, z), xm = site(L, (x + L - 1) % L, y, z);
                int yp = site(L, x, (y + 1) % L, z), ym = site(L, x, (y + L - 1) % L, z);
                int zp = site(L, x, y, (z + 1) % Lz), zm = site(L, x, y, (z + Lz - 1) % Lz);
                int *nb = o->nbr + 6 * s;
                nb[0] = xp;
                nb[1] = xm;
                nb[2] = yp;
                nb[3] = ym;
                nb[4] = zp;
                nb[5] = zm;
                int8_t *jn = o->Jn + 6 * s;
                jn[0] = o->J[0 * N + s];
                jn[1] = o->J[0 * N + xm];
                jn[2] = o->J[1 * N + s];
                jn[3] = o->J[1 * N + ym];
                jn[4] = dim == 3 ? o->J[2 * N + s] : 0;
                jn[5] = dim == 3 ? o->J[2 * N + zm] : 0;
                int32_t *jq = o->Jnq + 6 * s;
                jq[0] = o->Jq[0 * N + s];
                jq[1] = o->Jq[0 * N + xm];
                jq[2] = o->Jq[1 * N + s];
                jq[3] = o->Jq[1 * N + ym];
                jq[4] = dim == 3 ? o->Jq[2 * N + s] : 0;
                jq[5] = dim == 3 ? o->Jq[2 * N + zm] : 0;
                int c = colour_of(L, x, y, z);
                o->colour[s] = c;
                o->crank[s] = count[c]++;
            }
    init_population(o);
    return o;
}

orc_t *orc_create(int L, const int8_t *J, int64_t R, int64_t Rcap, const double *beta, int nT, int NS,
                  uint64_t seed, const uint8_t *overlap_steps, const int64_t *pop)
{
    if (!J) return NULL;
    return create(3, L, J, NULL, R, Rcap, beta, nT, NS, seed, overlap_steps, pop);
}

/* Real couplings: Jq int32 [3][N], J = Jq 2^-20, |J| < 8. */
orc_t *orc_create_real(int L, const int32_t *Jq, int64_t R, int64_t Rcap, const double *beta, int nT, int NS,
                       uint64_t seed, const uint8_t *overlap_steps, const int64_t *pop)
{
    if (!Jq) return NULL;
    return create(3, L, NULL, Jq, R, Rcap, beta, nT, NS, seed, overlap_steps, pop);
}

/* Real couplings on the periodic L^dim lattice, dim = 2 or 3: Jq int32
 * [dim][N]; 2 <= L <= 64 in 2D. */
orc_t *orc_create_real_dim(int dim, int L, const int32_t *Jq, int64_t R, int64_t Rcap, const double *beta, int nT,
                           int NS, uint64_t seed, const uint8_t *overlap_steps, const int64_t *pop)
{
    if (!Jq) return NULL;
    return create(dim, L, NULL, Jq, R, Rcap, beta, nT, NS, seed, overlap_steps, pop);
}

void orc_set_threads(orc_t *o, int n) { o->nthreads = n < 1 ? 1 : n; }

/* Metropolis acceptance thresholds for dE = 4, 8, 12 at inverse temperature
 * b: accept a move with dE > 0 when its uniform uint32 draw u is below
 * floor(exp(-b dE) 2^32), capped at 2^32 - 1.  beta = 0 accepts every move
 * (the flag), because 2^32 itself does not fit in 32 bits. */
void orc_thresholds(double b, uint32_t T[3], int *accept_all)
{
    *accept_all = (b == 0.0);
    for (int j = 0; j < 3; ++j) {
        double dE = 4.0 * (j + 1);
        double x = floor(exp(-b * dE) * 4294967296.0);
        T[j] = (x >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)x;
    }
}

/* exp(x) in binary32 for -23 <= x <= 0 (acceptance with real couplings).
 * Cody-Waite reduction x = n ln 2 + r, n = rint(x log2(e)), with ln 2 split
 * into a head of 16 significant bits (n ln2_hi is exact) and a tail; then
 * the Taylor polynomial of degree 7 in r (|r| <= ln(2)/2, truncation error
 * below 2^-27) by Horner's rule with fused multiply-adds, scaled by 2^n.
 * Every step is a correctly rounded binary32 operation, so any IEEE
 * implementation of the same steps returns the same bits. */
float orc_exp_f32(float x)
{
    const float log2e = 1.44269504f;
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = 1.42860677e-06f;
    float n = rintf(x * log2e);
    float r = fmaf(-n, ln2_hi, x);
    r = fmaf(-n, ln2_lo, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)n);
}

/* Metropolis acceptance of a move with dE > 0 (units of 2^-20) at
 * bq = beta 2^-20 rounded to binary32: x = -(bq dE) in binary32; rejected
 * for x < -23 (exp(x) 2^32 < 1); else accepted when e = exp(x) >= 1 or
 * u < floor(e 2^32). */
int orc_real_accept(float bq, int64_t dE, uint32_t u)
{
    float x = -(bq * (float)dE);
    if (x < -23.0f) return 0;
    float e = orc_exp_f32(x);
    if (e >= 1.0f) return 1;
    return u < (uint32_t)(e * 4294967296.0f);
}

/* beta_k 2^-20 rounded to binary32 (the scale is exact in binary64). */
static float real_beta(double b) { return (float)(b * 0x1p-20); }

/* N_S Metropolis sweeps of one replica at step k (Sec. II.B; checkerboard
 * order of Sec. III.A): colours ascending; inside a colour sites share no
 * bond, so visiting them lexicographically equals updating them at once.
 * S is the replica's configuration, *E its energy, r its row index (which
 * keys the draws together with k). */
static void sweep_one(const orc_t *o, int8_t *S, int64_t *Ep, int64_t r, int k, const uint32_t T[3],
                      int accept_all, int t0, int t1)
{
    int64_t E = *Ep;
    const float bq = real_beta(o->beta[k]);
    for (int t = t0; t < t1; ++t)
        for (int c = 0; c < o->ncol; ++c)
            for (int s = 0; s < o->N; ++s) {
                if (o->colour[s] != c) continue;
                const int *nb = o->nbr + 6 * s;
                int64_t h = 0;
                for (int d = 0; d < 2 * o->dim; ++d)
                    h += (o->gauss ? (int64_t)o->Jnq[6 * s + d] : (int64_t)o->Jn[6 * s + d]) * S[nb[d]];
                int64_t dE = 2 * S[s] * h;
                int i = o->crank[s];
                uint32_t u = draw(o->seed, ((uint32_t)c << 24) | (uint32_t)(i >> 2), (uint32_t)r,
                                  (uint32_t)k, TAG_SWEEP | (uint32_t)t, i & 3);
                int accept = accept_all || dE <= 0 ||
                             (o->gauss ? orc_real_accept(bq, dE, u) : u < T[dE / 4 - 1]);
                if (accept) {
                    S[s] = (int8_t)-S[s];
                    E += dE;
                }
            }
    *Ep = E;
}

/* Sweeps t0 .. t1-1 of replica r at the current step. */
static void sweep_replica(orc_t *o, int64_t r, const uint32_t T[3], int accept_all, int t0, int t1)
{
    sweep_one(o, o->spin + r * o->N, &o->E[r], r, o->k, T, accept_all, t0, t1);
}

/* ------------------------------------------------------------------------ */
/* Isoenergetic cluster moves (Sec. IV)                                      */
/* ------------------------------------------------------------------------ */
/* Keyed pseudo-random permutation of [0, n): a balanced Feistel network on
 * 2h-bit words (4^h >= n) of four rounds, (l, r) -> (r, l ^ F_j(r)), with
 * F_j(r) = word 0 of Philox at counter (r, j, k, TAG_ICM | round) masked to
 * h bits, applied repeatedly from i until the value falls in [0, n) (cycle
 * walking; it ends because i itself lies on the cycle). */
uint32_t orc_icm_perm(uint64_t seed, uint32_t i, uint32_t n, int k, int round)
{
    int h = 0;
    while (((uint64_t)1 << (2 * h)) < (uint64_t)n) ++h;
    const uint32_t mask = h == 0 ? 0u : (uint32_t)(((uint64_t)1 << h) - 1);
    uint32_t x = i;
    do {
        uint32_t l = h == 0 ? 0u : x >> h, r = x & mask;
        for (int j = 0; j < 4; ++j) {
            uint32_t f = draw(seed, r, (uint32_t)j, (uint32_t)k, TAG_ICM | (uint32_t)round, 0) & mask;
            uint32_t t = l ^ f;
            l = r;
            r = t;
        }
        x = h == 0 ? 0u : ((l << h) | r);
    } while (x >= n);
    return x;
}

/* One ICM update of the pair (Sa, Sb), pair index j of round `round` at step
 * k: the sector of sites where the replicas differ (q = -1) or agree
 * (q = +1), whichever has fewer sites (the differing one on a tie); the
 * m-th site of that sector in lexicographic order with
 * m = floor(u * count / 2^32), u = word 0 of Philox at counter
 * (j, 4, k, TAG_ICM | round); its island, the sites of the sector connected
 * to it by lattice bonds, flipped in both replicas.  Returns the island
 * size (0: empty sector). */
int orc_icm_pair(const orc_t *o, int8_t *Sa, int8_t *Sb, uint32_t j, int k, int round)
{
    const int N = o->N;
    int ndiff = 0;
    for (int s = 0; s < N; ++s) ndiff += Sa[s] != Sb[s];
    const int want_diff = ndiff <= N - ndiff;
    const int cnt = want_diff ? ndiff : N - ndiff;
    if (cnt == 0) return 0;
    const uint32_t u = draw(o->seed, j, 4u, (uint32_t)k, TAG_ICM | (uint32_t)round, 0);
    const int m = (int)(((uint64_t)u * (uint64_t)cnt) >> 32);
    int s0 = -1;
    for (int s = 0, seen = 0; s < N; ++s)
        if ((Sa[s] != Sb[s]) == want_diff) {
            if (seen == m) {
                s0 = s;
                break;
            }
            ++seen;
        }
    uint8_t *in = (uint8_t *)calloc((size_t)N, 1);
    int *queue = (int *)malloc(sizeof(int) * (size_t)N);
    if (!in || !queue) {
        free(in);
        free(queue);
        return -1;
    }
    int head = 0, tail = 0;
    queue[tail++] = s0;
    in[s0] = 1;
    while (head < tail) {
        const int s = queue[head++];
        for (int d = 0; d < 2 * o->dim; ++d) {
            const int t = o->nbr[6 * s + d];
            if (!in[t] && (Sa[t] != Sb[t]) == want_diff) {
                in[t] = 1;
                queue[tail++] = t;
            }
        }
    }
    for (int q = 0; q < tail; ++q) {
        Sa[queue[q]] = (int8_t)-Sa[queue[q]];
        Sb[queue[q]] = (int8_t)-Sb[queue[q]];
    }
    free(in);
    free(queue);
    return tail;
}

/* The ICM rounds of the current step: round rd pairs rows
 * perm(2j) and perm(2j+1), j < floor(R_k/2); energies are recomputed. */
static int icm_step(orc_t *o)
{
    const uint32_t n = (uint32_t)o->Rk;
    for (int rd = 0; rd < o->icm_rounds; ++rd)
        for (uint32_t j = 0; j < n / 2; ++j) {
            const uint32_t a = orc_icm_perm(o->seed, 2 * j, n, o->k, rd);
            const uint32_t b = orc_icm_perm(o->seed, 2 * j + 1, n, o->k, rd);
            if (orc_icm_pair(o, o->spin + (size_t)a * o->N, o->spin + (size_t)b * o->N, j, o->k, rd) < 0)
                return ORC_ERR_NOMEM;
        }
    for (int64_t r = 0; r < o->Rk; ++r) o->E[r] = energy(o, o->spin + r * o->N);
    return ORC_OK;
}

void orc_set_icm(orc_t *o, int rounds, double beta_min)
{
    o->icm_rounds = rounds < 0 ? 0 : rounds;
    o->icm_beta_min = beta_min;
}

/* Pairwise summation tree over n leaves (n a power of two): level by level,
 * node i of the next level is left child 2i plus right child 2i+1. */
static double pairwise_tree(double *a, int64_t n)
{
    while (n > 1) {
        for (int64_t i = 0; i < n / 2; ++i) a[i] = a[2 * i] + a[2 * i + 1];
        n /= 2;
    }
    return a[0];
}

static int64_t pow2_at_least(int64_t n)
{
    int64_t p = 1;
    while (p < n) p *= 2;
    return p;
}

/* Measurements at step k (Sec. II.B, Eq. (2); Sec. V.A, Eq. (9)). */
static int measure(orc_t *o)
{
    int k = o->k, N = o->N;
    int64_t sumE = 0;
    __int128 sumE2 = 0;
    int64_t Emin = o->E[0], Emax = o->E[0];
    for (int64_t r = 0; r < o->Rk; ++r) {
        int64_t e = o->E[r];
        sumE += e;
        sumE2 += (__int128)e * e;
        if (o->E[r] < Emin) Emin = o->E[r];
        if (o->E[r] > Emax) Emax = o->E[r];
    }
    o->o_R[k] = o->Rk;
    o->o_sumE[k] = sumE;
    o->o_sumE2[k] = sumE2;
    o->o_Emin[k] = Emin;
    o->o_Emax[k] = Emax;
    o->o_lnZ[k] = o->lnZ;

    /* Family term sum_i n_i ln n_i over the initial replicas i (families),
     * n_i = number of descendants of i; summed by the pairwise tree over
     * family ids 0 .. P-1 (P = smallest power of two >= R). */
    int64_t P = pow2_at_least(o->R);
    uint32_t *cnt = (uint32_t *)calloc((size_t)o->R, sizeof(uint32_t));
    double *leaf = (double *)calloc((size_t)P, sizeof(double));
    if (!cnt || !leaf) {
        free(cnt);
        free(leaf);
        return ORC_ERR_NOMEM;
    }
    for (int64_t r = 0; r < o->Rk; ++r) cnt[o->fam[r]]++;
    for (int64_t f = 0; f < o->R; ++f)
        leaf[f] = cnt[f] > 0 ? (double)cnt[f] * log((double)cnt[f]) : 0.0;
    o->o_T[k] = pairwise_tree(leaf, P);
    free(cnt);
    free(leaf);

    /* Spin overlap at selected steps (Sec. V.A): replica r is paired with
     * r + floor(R_k / 2); Q = sum_s S_s S'_s, histogram over Q + N. */
    if (o->ovl[k]) {
        int64_t *q = o->o_q + (size_t)k * (2 * N + 1);
        int64_t h = o->Rk / 2;
        for (int64_t r = 0; r < h; ++r) {
            const int8_t *a = o->spin + r * N, *b = o->spin + (r + h) * N;
            int Q = 0;
            for (int s = 0; s < N; ++s) Q += a[s] * b[s];
            q[Q + N]++;
        }
    }
    return ORC_OK;
}

/* Stable copy of the population by the copy numbers o->ncopy (source order,
 * so families stay contiguous), then swap of the buffers. */
static void copy_population(orc_t *o)
{
    int N = o->N;
    int64_t d = 0;
    for (int64_t r = 0; r < o->Rk; ++r)
        for (uint32_t j = 0; j < o->ncopy[r]; ++j, ++d) {
            memcpy(o->spin2 + d * N, o->spin + r * N, (size_t)N);
            o->E2[d] = o->E[r];
            o->fam2[d] = o->fam[r];
        }
    int8_t *ts = o->spin;
    o->spin = o->spin2;
    o->spin2 = ts;
    int64_t *te = o->E;
    o->E = o->E2;
    o->E2 = te;
    uint32_t *tf = o->fam;
    o->fam = o->fam2;
    o->fam2 = tf;
}

/* Resampling with real couplings (Sec. II.B): replica i's weight relative to
 * the lowest energy is w_i = exp(-dbeta (E_i - E_min)); with D_i = E_i - E_min
 * in units of 2^-20 it is the product, over the set bits b of D_i in
 * ascending order, of pw[b] = exp(-dbeta 2^(b-20)) (libm).  S is the
 * pairwise tree over the replica rows 0 .. P-1 (P the smallest power of two
 * >= R_k, zero leaves beyond R_k); tau_i = R' w_i / S and the copy numbers
 * follow as for +-1 couplings. */
static int resample_real(orc_t *o, double dbeta)
{
    int k = o->k;
    int64_t Emin = o->o_Emin[k];
    double pw[40];
    for (int b = 0; b < 40; ++b) pw[b] = exp(-dbeta * ldexp(1.0, b - 20));
    int64_t P = pow2_at_least(o->Rk);
    double *w = (double *)malloc(sizeof(double) * (size_t)o->Rk);
    double *leaf = (double *)calloc((size_t)P, sizeof(double));
    if (!w || !leaf) {
        free(w);
        free(leaf);
        return ORC_ERR_NOMEM;
    }
    for (int64_t r = 0; r < o->Rk; ++r) {
        int64_t D = o->E[r] - Emin;
        double x = 1.0;
        for (int b = 0; b < 40; ++b)
            if ((D >> b) & 1) x = x * pw[b];
        w[r] = x;
        leaf[r] = x;
    }
    double S = pairwise_tree(leaf, P);
    int64_t Rn = 0;
    for (int64_t r = 0; r < o->Rk; ++r) {
        double tau = ((double)o->Rt[k + 1] * w[r]) / S;
        double fl = floor(tau);
        uint32_t B = (uint32_t)fl;
        uint32_t F = (uint32_t)floor((tau - fl) * 4294967296.0);
        uint32_t u = draw(o->seed, 0u, (uint32_t)r, (uint32_t)k, TAG_RESAMPLE, 0);
        o->ncopy[r] = B + (u < F ? 1u : 0u);
        Rn += o->ncopy[r];
    }
    free(w);
    free(leaf);
    if (Rn > o->Rcap) return ORC_ERR_CAPACITY;
    if (Rn == 0) return ORC_ERR_EXTINCT;
    copy_population(o);
    /* free-energy perturbation as for +-1 couplings, E_min in energy units */
    double lnQ = (-dbeta * ((double)Emin * 0x1p-20)) + log(S) - log((double)o->Rk);
    o->o_S[k] = S;
    o->o_lnQ[k] = lnQ;
    o->lnZ = o->lnZ + lnQ;
    o->Rk = Rn;
    return ORC_OK;
}

/* Resampling from beta_k to beta_{k+1} (Sec. II.B).  The mean number of
 * copies of replica i is tau_i = R' exp[-(beta'-beta) E_i] / sum_j exp[...],
 * so that the expected new population is the nominal R' = R(beta_{k+1})
 * (constant unless a population schedule was given, Sec. III.D); replica i
 * gets floor(tau_i) copies plus one more with probability frac(tau_i).
 * Copies keep source order (families stay contiguous). */
static int resample(orc_t *o)
{
    int k = o->k, N = o->N;
    double dbeta = o->beta[k + 1] - o->beta[k];
    if (o->gauss) return resample_real(o, dbeta);
    int64_t Emin = o->o_Emin[k], Emax = o->o_Emax[k];
    int64_t M = (Emax - Emin) / 2; /* energies differ by multiples of 2 */
    int64_t P = pow2_at_least(M + 1);
    int64_t *hist = (int64_t *)calloc((size_t)(M + 1), sizeof(int64_t));
    double *w = (double *)malloc(sizeof(double) * (size_t)(M + 1));
    double *leaf = (double *)calloc((size_t)P, sizeof(double));
    uint32_t *B = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(M + 1));
    uint32_t *F = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(M + 1));
    if (!hist || !w || !leaf || !B || !F) {
        free(hist);
        free(w);
        free(leaf);
        free(B);
        free(F);
        return ORC_ERR_NOMEM;
    }
    for (int64_t r = 0; r < o->Rk; ++r) hist[(o->E[r] - Emin) / 2]++;

    /* Level weights w[m] = exp(-dbeta (E - E_min)) = rho^m, rho = exp(-2 dbeta),
     * formed as the product of rho^(2^b) over the set bits b of m, ascending. */
    double rho = exp(-2.0 * dbeta);
    double pw[64];
    pw[0] = rho;
    for (int b = 1; b < 64; ++b) pw[b] = pw[b - 1] * pw[b - 1];
    for (int64_t m = 0; m <= M; ++m) {
        double x = 1.0;
        for (int b = 0; b < 63; ++b)
            if ((m >> b) & 1) x = x * pw[b];
        w[m] = x;
    }
    for (int64_t m = 0; m <= M; ++m) leaf[m] = (double)hist[m] * w[m];
    double S = pairwise_tree(leaf, P);

    for (int64_t m = 0; m <= M; ++m) {
        double tau = ((double)o->Rt[k + 1] * w[m]) / S;
        double fl = floor(tau);
        B[m] = (uint32_t)fl;
        F[m] = (uint32_t)floor((tau - fl) * 4294967296.0);
    }

    int64_t Rn = 0;
    for (int64_t r = 0; r < o->Rk; ++r) {
        int64_t m = (o->E[r] - Emin) / 2;
        uint32_t u = draw(o->seed, 0u, (uint32_t)r, (uint32_t)k, TAG_RESAMPLE, 0);
        o->ncopy[r] = B[m] + (u < F[m] ? 1u : 0u);
        Rn += o->ncopy[r];
    }
    free(hist);
    free(w);
    free(leaf);
    free(B);
    free(F);
    if (Rn > o->Rcap) return ORC_ERR_CAPACITY;
    if (Rn == 0) return ORC_ERR_EXTINCT;

    int64_t d = 0;
    for (int64_t r = 0; r < o->Rk; ++r)
        for (uint32_t j = 0; j < o->ncopy[r]; ++j, ++d) {
            memcpy(o->spin2 + d * N, o->spin + r * N, (size_t)N);
            o->E2[d] = o->E[r];
            o->fam2[d] = o->fam[r];
        }
    int8_t *ts = o->spin;
    o->spin = o->spin2;
    o->spin2 = ts;
    int64_t *te = o->E;
    o->E = o->E2;
    o->E2 = te;
    uint32_t *tf = o->fam;
    o->fam = o->fam2;
    o->fam2 = tf;

    /* Free-energy perturbation: Q_k = (1/R_k) sum_i exp(-dbeta E_i)
     * = exp(-dbeta E_min) S / R_k, and ln Z_{k+1} = ln Z_k + ln Q_k. */
    double lnQ = (-dbeta * (double)Emin) + log(S) - log((double)o->Rk);
    o->o_S[k] = S;
    o->o_lnQ[k] = lnQ;
    o->lnZ = o->lnZ + lnQ;
    o->Rk = Rn;
    return ORC_OK;
}

/* Run up to n_steps temperature steps (n_steps < 0: to the end).  A step k
 * is: N_S sweeps at beta_k, measurement, and (k < nT-1) resampling. */
int orc_run(orc_t *o, int n_steps)
{
    if (!o) return ORC_ERR_INVALID;
    int done = 0;
    while (o->k < o->nT && (n_steps < 0 || done < n_steps)) {
        uint32_t T[3];
        int all;
        orc_thresholds(o->beta[o->k], T, &all);
        /* with ICM (steps after a resampling): N_S/2 sweeps, the cluster
         * updates, the remaining sweeps */
        const int icm = o->icm_rounds > 0 && o->k >= 1 && o->beta[o->k] >= o->icm_beta_min;
        const int t_mid = icm ? o->NS / 2 : o->NS;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(o->nthreads)
#endif
        for (int64_t r = 0; r < o->Rk; ++r) sweep_replica(o, r, T, all, 0, t_mid);
        if (icm) {
            int sti = icm_step(o);
            if (sti != ORC_OK) return sti;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(o->nthreads)
#endif
            for (int64_t r = 0; r < o->Rk; ++r) sweep_replica(o, r, T, all, t_mid, o->NS);
        }
        int st = measure(o);
        if (st != ORC_OK) return st;
        if (o->k < o->nT - 1) {
            st = resample(o);
            if (st != ORC_OK) return st;
        }
        o->k += 1;
        done += 1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Accessors for the ctypes wrapper                                          */
/* ------------------------------------------------------------------------ */
int orc_step(const orc_t *o) { return o->k; }
int64_t orc_population(const orc_t *o) { return o->Rk; }
int orc_num_spins(const orc_t *o) { return o->N; }
double orc_lnZ(const orc_t *o) { return o->lnZ; }

/* Per-step records with the exact sum of E^2 as two 64-bit halves:
 * ints[k][6] = R_k, sum E, low and high 64 bits of sum E^2, E_min, E_max. */
int orc_records_wide(const orc_t *o, int64_t *ints)
{
    for (int k = 0; k < o->nT; ++k) {
        unsigned __int128 v = (unsigned __int128)o->o_sumE2[k];
        ints[6 * k + 0] = o->o_R[k];
        ints[6 * k + 1] = o->o_sumE[k];
        ints[6 * k + 2] = (int64_t)(uint64_t)v;
        ints[6 * k + 3] = (int64_t)(uint64_t)(v >> 64);
        ints[6 * k + 4] = o->o_Emin[k];
        ints[6 * k + 5] = o->o_Emax[k];
    }
    return ORC_OK;
}

/* Per-step records: ints[k][5] = R_k, sum E, sum E^2, E_min, E_max;
 * dbl[k][4] = S_k (normaliser), family term T_k, ln Q_k, ln Z_k. */
int orc_records(const orc_t *o, int64_t *ints, double *dbl, int64_t *qhist)
{
    for (int k = 0; k < o->nT; ++k) {
        ints[5 * k + 0] = o->o_R[k];
        ints[5 * k + 1] = o->o_sumE[k];
        ints[5 * k + 2] = (int64_t)o->o_sumE2[k];
        ints[5 * k + 3] = o->o_Emin[k];
        ints[5 * k + 4] = o->o_Emax[k];
        dbl[4 * k + 0] = o->o_S[k];
        dbl[4 * k + 1] = o->o_T[k];
        dbl[4 * k + 2] = o->o_lnQ[k];
        dbl[4 * k + 3] = o->o_lnZ[k];
    }
    if (qhist) memcpy(qhist, o->o_q, sizeof(int64_t) * (size_t)o->nT * (2 * o->N + 1));
    return ORC_OK;
}

/* Current population: spins [R_k][N] int8 +-1 lexicographic, E, family. */
int orc_get_state(const orc_t *o, int8_t *spins, int32_t *E, uint32_t *fam)
{
    memcpy(spins, o->spin, (size_t)o->Rk * o->N);
    for (int64_t r = 0; r < o->Rk; ++r) E[r] = (int32_t)o->E[r];
    memcpy(fam, o->fam, sizeof(uint32_t) * (size_t)o->Rk);
    return ORC_OK;
}

/* The same with 64-bit energies (units of 2^-20 for real couplings). */
int orc_get_state64(const orc_t *o, int8_t *spins, int64_t *E, uint32_t *fam)
{
    memcpy(spins, o->spin, (size_t)o->Rk * o->N);
    memcpy(E, o->E, sizeof(int64_t) * (size_t)o->Rk);
    memcpy(fam, o->fam, sizeof(uint32_t) * (size_t)o->Rk);
    return ORC_OK;
}

/* Replace the population (checkpoint resume / step-wise parity).  Energies
 * are recomputed from the spins with Eq. (1). */
int orc_set_state(orc_t *o, int k, int64_t Rk, const int8_t *spins, const uint32_t *fam, double lnZ)
{
    if (k < 0 || k >= o->nT || Rk < 1 || Rk > o->Rcap) return ORC_ERR_INVALID;
    for (int64_t i = 0; i < Rk * o->N; ++i)
        if (spins[i] != 1 && spins[i] != -1) return ORC_ERR_INVALID;
    for (int64_t r = 0; r < Rk; ++r)
        if (fam[r] >= (uint64_t)o->R) return ORC_ERR_INVALID;
    memcpy(o->spin, spins, (size_t)Rk * o->N);
    memcpy(o->fam, fam, sizeof(uint32_t) * (size_t)Rk);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(o->nthreads)
#endif
    for (int64_t r = 0; r < Rk; ++r) o->E[r] = energy(o, o->spin + r * o->N);
    o->Rk = Rk;
    o->k = k;
    o->lnZ = lnZ;
    return ORC_OK;
}

/* Energy of arbitrary configurations of this instance (Eq. (1)). */
int orc_energies(const orc_t *o, const int8_t *spins, int64_t n, int32_t *E)
{
    for (int64_t r = 0; r < n; ++r) E[r] = (int32_t)energy(o, spins + r * o->N);
    return ORC_OK;
}

int orc_energies64(const orc_t *o, const int8_t *spins, int64_t n, int64_t *E)
{
    for (int64_t r = 0; r < n; ++r) E[r] = energy(o, spins + r * o->N);
    return ORC_OK;
}

/* Colour and colour rank of every site, for tests of the colouring. */
int orc_colouring(const orc_t *o, int32_t *colour, int32_t *crank)
{
    for (int s = 0; s < o->N; ++s) {
        colour[s] = o->colour[s];
        crank[s] = o->crank[s];
    }
    return o->ncol;
}

/* Neighbour table [N][6] (+x, -x, +y, -y, +z, -z). */
int orc_neighbours(const orc_t *o, int32_t *nb)
{
    for (int i = 0; i < 6 * o->N; ++i) nb[i] = o->nbr[i];
    return ORC_OK;
}

/* Derived observables per step k (Sec. II.B, Eq. (2); Sec. V.A, Eq. (9)),
 * out[k][12] = beta, R_k, <E>, <E>/N, C_V, ln Q_k, ln Z_k, beta F_k, f_k,
 * S_f, rho_s, and the overlap Binder cumulant g_SG (NaN when the overlap was
 * not measured at k).  Definitions:
 *   <E> = sum E / R_k;  C_V = beta^2 var(E) / N with the variance taken
 *   exactly in integers, (R_k sum E^2 - (sum E)^2) / R_k^2 (for real
 *   couplings the integer sums are in units of 2^-20 and 2^-40, scaled
 *   after the division);
 *   beta F = -ln Z;  f = -ln Z / (beta N) (NaN at beta = 0);
 *   S_f = ln R_k - (1/R_k) sum_i n_i ln n_i  (= -sum_i nu_i ln nu_i);
 *   rho_s = R_k / e^{S_f} with the local R_k;
 *   q = Q / N, <q^p> = sum_Q h[Q] q^p / sum_Q h[Q] in ascending Q,
 *   g_SG = (3 - <q^4>/<q^2>^2) / 2.
 * ovl_out[k][3] = <|q|>, <q^2>, <q^4> (NaN when not measured). */
int orc_observables(const orc_t *o, double *out, double *ovl_out)
{
    int N = o->N;
    for (int k = 0; k < o->nT; ++k) {
        double *v = out + 12 * k;
        double b = o->beta[k];
        int64_t Rk = o->o_R[k];
        for (int i = 0; i < 12; ++i) v[i] = NAN;
        for (int i = 0; i < 3; ++i) ovl_out[3 * k + i] = NAN;
        v[0] = b;
        if (Rk <= 0) continue;
        double R = (double)Rk;
        /* energies in units of 2^-20 for real couplings (exact scalings) */
        double sc = o->gauss ? 0x1p-20 : 1.0;
        double meanE = ((double)o->o_sumE[k] * sc) / R;
        __int128 num = (__int128)Rk * o->o_sumE2[k] - (__int128)o->o_sumE[k] * (__int128)o->o_sumE[k];
        double var = ((double)num / (R * R)) * (sc * sc);
        v[1] = R;
        v[2] = meanE;
        v[3] = meanE / (double)N;
        v[4] = (b * b) * var / (double)N;
        v[5] = (k < o->nT - 1) ? o->o_lnQ[k] : NAN;
        v[6] = o->o_lnZ[k];
        v[7] = -o->o_lnZ[k];
        v[8] = (b > 0.0) ? -o->o_lnZ[k] / (b * (double)N) : NAN;
        double Sf = log(R) - o->o_T[k] / R;
        v[9] = Sf;
        v[10] = R / exp(Sf);
        if (o->ovl[k]) {
            const int64_t *h = o->o_q + (size_t)k * (2 * N + 1);
            int64_t n = 0;
            double m1 = 0.0, m2 = 0.0, m4 = 0.0;
            for (int Q = -N; Q <= N; ++Q) {
                int64_t c = h[Q + N];
                if (c == 0) continue;
                double q = (double)Q / (double)N;
                n += c;
                m1 += (double)c * fabs(q);
                m2 += (double)c * (q * q);
                m4 += (double)c * ((q * q) * (q * q));
            }
            if (n > 0) {
                m1 /= (double)n;
                m2 /= (double)n;
                m4 /= (double)n;
                ovl_out[3 * k + 0] = m1;
                ovl_out[3 * k + 1] = m2;
                ovl_out[3 * k + 2] = m4;
                v[11] = 0.5 * (3.0 - m4 / (m2 * m2));
            }
        }
    }
    return ORC_OK;
}

/* Sweeps of selected replicas at step k, for checks that sample a large
 * population: rows[i] is the replica's row index (it keys the draws) and
 * spins[i][N] (int8 +-1) is overwritten by its configuration after the N_S
 * sweeps of step k; E[i] receives its energy.  The handle's population is
 * untouched. */
int orc_sweep_rows64(orc_t *o, int k, int64_t n, const int64_t *rows, int8_t *spins, int64_t *E);

int orc_sweep_rows(orc_t *o, int k, int64_t n, const int64_t *rows, int8_t *spins, int32_t *E)
{
    int64_t *E64 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!E64) return ORC_ERR_NOMEM;
    int st = orc_sweep_rows64(o, k, n, rows, spins, E64);
    for (int64_t i = 0; i < n; ++i) E[i] = (int32_t)E64[i];
    free(E64);
    return st;
}

/* The same with 64-bit energies (units of 2^-20 for real couplings). */
int orc_sweep_rows64(orc_t *o, int k, int64_t n, const int64_t *rows, int8_t *spins, int64_t *E)
{
    if (k < 0 || k >= o->nT || n < 0) return ORC_ERR_INVALID;
    uint32_t T[3];
    int all;
    orc_thresholds(o->beta[k], T, &all);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(o->nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int8_t *S = spins + i * o->N;
        E[i] = energy(o, S);
        sweep_one(o, S, &E[i], rows[i], k, T, all, 0, o->NS);
    }
    return ORC_OK;
}

/* Measurement and resampling of the current population at the current step
 * without sweeping it first (the population is taken as the post-sweep
 * state of that step), then advance to the next step. */
int orc_measure_resample(orc_t *o)
{
    if (o->k >= o->nT) return ORC_ERR_STATE;
    int st = measure(o);
    if (st != ORC_OK) return st;
    if (o->k < o->nT - 1) {
        st = resample(o);
        if (st != ORC_OK) return st;
    }
    o->k += 1;
    return ORC_OK;
}
