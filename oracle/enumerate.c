/*
 * enumerate.c -- exact thermodynamics of tiny +-J Edwards-Anderson instances
 * by visiting every spin configuration.
 *
 * TEST INFRASTRUCTURE ONLY: the exact values that pin the PAMC oracle
 * (partition function, mean energy, specific heat, overlap distribution).
 *
 * Hamiltonian of Sec. II.A, Eq. (1), H = -sum_<ij> J_ij S_i S_j on the
 * periodic L^3 lattice.  The 3N bonds are listed explicitly: bond (s, d)
 * joins s and s + e_d with coupling J[d][s], so for L = 2 two distinct bonds
 * join each pair of x-, y- or z-neighbours.  Written independently of the
 * PAMC oracle's neighbour tables.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int a, b, j;
} bond_t;

static int build_bonds(int L, const int8_t *J, bond_t *bonds)
{
    int N = L * L * L, n = 0;
    for (int d = 0; d < 3; ++d)
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int s = x + L * (y + L * z);
                    int xx = x, yy = y, zz = z;
                    if (d == 0) xx = (x + 1) % L;
                    if (d == 1) yy = (y + 1) % L;
                    if (d == 2) zz = (z + 1) % L;
                    bonds[n].a = s;
                    bonds[n].b = xx + L * (yy + L * zz);
                    bonds[n].j = J[d * N + s];
                    ++n;
                }
    return n;
}

/* Density of states g[(E + 3N) / 2] over all 2^N configurations, by a Gray
 * code walk: consecutive configurations differ in the spin at the lowest set
 * bit of the step index, and the energy is updated by the change of the
 * bonds touching that spin.  N <= 30. */
int enum_dos(int L, const int8_t *J, int64_t *g)
{
    int N = L * L * L;
    if (N > 30) return -1;
    int nb = 3 * N;
    bond_t *bonds = (bond_t *)malloc(sizeof(bond_t) * nb);
    int *deg = (int *)calloc(N, sizeof(int));
    int *adj = (int *)malloc(sizeof(int) * 6 * N); /* bond indices per site */
    int8_t *S = (int8_t *)malloc(N);
    if (!bonds || !deg || !adj || !S) {
        free(bonds);
        free(deg);
        free(adj);
        free(S);
        return -2;
    }
    build_bonds(L, J, bonds);
    for (int i = 0; i < nb; ++i) {
        adj[6 * bonds[i].a + deg[bonds[i].a]++] = i;
        adj[6 * bonds[i].b + deg[bonds[i].b]++] = i;
    }
    for (int i = 0; i <= 3 * N; ++i) g[i] = 0;
    int64_t E = 0;
    for (int s = 0; s < N; ++s) S[s] = -1;
    for (int i = 0; i < nb; ++i) E -= bonds[i].j * S[bonds[i].a] * S[bonds[i].b];
    g[(E + 3 * N) / 2]++;
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t step = 1; step < total; ++step) {
        int s = __builtin_ctzll(step);
        int64_t before = 0;
        for (int q = 0; q < 6; ++q) {
            const bond_t *b = &bonds[adj[6 * s + q]];
            before -= b->j * S[b->a] * S[b->b];
        }
        /* flipping S_s negates every bond term touching s */
        E += -2 * before;
        S[s] = (int8_t)-S[s];
        g[(E + 3 * N) / 2]++;
    }
    free(bonds);
    free(deg);
    free(adj);
    free(S);
    return 0;
}

/* Energy of every configuration (bit s of the index set means S_s = +1),
 * directly from the bond list.  N <= 20. */
int enum_energies(int L, const int8_t *J, int32_t *E)
{
    int N = L * L * L;
    if (N > 20) return -1;
    int nb = 3 * N;
    bond_t *bonds = (bond_t *)malloc(sizeof(bond_t) * nb);
    if (!bonds) return -2;
    build_bonds(L, J, bonds);
    for (uint64_t c = 0; c < ((uint64_t)1 << N); ++c) {
        int32_t e = 0;
        for (int i = 0; i < nb; ++i) {
            int sa = ((c >> bonds[i].a) & 1) ? 1 : -1;
            int sb = ((c >> bonds[i].b) & 1) ? 1 : -1;
            e -= bonds[i].j * sa * sb;
        }
        E[c] = e;
    }
    free(bonds);
    return 0;
}

/* Exact distribution of the overlap Q = sum_s S^a_s S^b_s between two
 * independent Boltzmann-distributed configurations at inverse temperature
 * beta: P[Q + N] = sum_{a,b: Q(a,b) = Q} e^{-beta (E_a + E_b)} / Z^2.
 * N <= 12. */
int enum_overlap(int L, const int8_t *J, double beta, double *P)
{
    int N = L * L * L;
    if (N > 12) return -1;
    uint64_t nc = (uint64_t)1 << N;
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * nc);
    double *w = (double *)malloc(sizeof(double) * nc);
    if (!E || !w) {
        free(E);
        free(w);
        return -2;
    }
    enum_energies(L, J, E);
    int32_t Emin = E[0];
    for (uint64_t c = 0; c < nc; ++c)
        if (E[c] < Emin) Emin = E[c];
    double Z = 0.0;
    for (uint64_t c = 0; c < nc; ++c) {
        w[c] = exp(-beta * (double)(E[c] - Emin));
        Z += w[c];
    }
    for (int q = 0; q <= 2 * N; ++q) P[q] = 0.0;
    for (uint64_t a = 0; a < nc; ++a)
        for (uint64_t b = 0; b < nc; ++b) {
            int Q = N - 2 * __builtin_popcountll(a ^ b);
            P[Q + N] += w[a] * w[b];
        }
    for (int q = 0; q <= 2 * N; ++q) P[q] /= Z * Z;
    free(E);
    free(w);
    return 0;
}

/* Energies, in units of 2^-20, of all 2^N configurations of an instance with
 * real couplings Jq [3][N] (J = Jq 2^-20): configuration c has S_s = +1 when
 * bit s of c is set.  Each energy is the plain sum over the 3N bonds,
 * Eq. (1).  N <= 24. */
int enum_energies_real(int L, const int32_t *Jq, int64_t *E)
{
    int N = L * L * L;
    if (N > 24) return -1;
    int nb = 3 * N;
    int *a = (int *)malloc(sizeof(int) * nb), *b = (int *)malloc(sizeof(int) * nb);
    int64_t *j = (int64_t *)malloc(sizeof(int64_t) * nb);
    if (!a || !b || !j) {
        free(a);
        free(b);
        free(j);
        return -2;
    }
    int n = 0;
    for (int d = 0; d < 3; ++d)
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int s = x + L * (y + L * z);
                    int xx = d == 0 ? (x + 1) % L : x, yy = d == 1 ? (y + 1) % L : y, zz = d == 2 ? (z + 1) % L : z;
                    a[n] = s;
                    b[n] = xx + L * (yy + L * zz);
                    j[n] = Jq[d * N + s];
                    ++n;
                }
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t c = 0; c < total; ++c) {
        int64_t e = 0;
        for (int i = 0; i < nb; ++i) {
            int sa = ((c >> a[i]) & 1) ? 1 : -1, sb = ((c >> b[i]) & 1) ? 1 : -1;
            e -= j[i] * sa * sb;
        }
        E[c] = e;
    }
    free(a);
    free(b);
    free(j);
    return 0;
}
