/* Host sanitizer run of the CPU oracle (test infrastructure): built with
 * gcc -fsanitize=address,undefined together with oracle/scqmc_oracle.c by
 * tests/test_oracle_sanitize.py, it drives every public entry point of the
 * oracle on a small seeded system (1 core, 3 active, 3 virtual orbitals,
 * 2 + 2 electrons, every active-space determinant in the reference) and
 * checks that the results are finite.  Any out-of-bounds access, leak or
 * undefined operation aborts the run with a sanitizer report. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc orc_t;
orc_t *orc_create(int n_orb, int n_core, int n_act, int n_a, int n_b);
void orc_destroy(orc_t *o);
int64_t orc_n_classes(const orc_t *o);
int orc_set_integrals_chol(orc_t *o, const double *h1, const double *B, int n_chol, double e_const);
int orc_set_reference(orc_t *o, int64_t n, const uint64_t *dets, const double *coeff);
int orc_set_coeffs(orc_t *o, double c0, const double *c_cls, int64_t n);
int orc_set_dyall(orc_t *o, const double *eps_v, double e0);
void orc_set_options(orc_t *o, double eps_screen, int mode);
double orc_psi(const orc_t *o, const uint64_t *m);
int64_t orc_neighbors(const orc_t *o, const uint64_t *det, int64_t cap, uint64_t *out_dets, int8_t *out_phase,
                      double *out_h, double *out_psi, double *out_hd, int64_t *out_cls);
int orc_eval(const orc_t *o, int64_t n, const uint64_t *dets, double *eloc, double *psi, double *gamma,
             double *eloc_d, int64_t *cls, double *sabs, double *kappa, int nthreads);
int64_t orc_run(const orc_t *o, int64_t W, uint64_t *dets, double *psi_out, uint64_t seed, int64_t step0,
                int64_t n_steps, int64_t burn_in, int64_t wid0, double *wsum, double *csum, int nthreads);
int64_t orc_det_hamiltonian(const orc_t *o, int64_t n, const uint64_t *dets, int64_t cap, int64_t *rows,
                            int64_t *cols, double *vals);
double orc_reference_energy(const orc_t *o);
void orc_reference_rdm1(const orc_t *o, double *gamma);
void orc_traffic(const orc_t *o, const uint64_t *n, int64_t out[5]);

#define N 7
#define NC 1
#define NA 3
#define L 5

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) {   /* xorshift64*, uniform in [-0.5, 0.5) */
    rng_state ^= rng_state >> 12; rng_state ^= rng_state << 25; rng_state ^= rng_state >> 27;
    return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1.0p-53 - 0.5;
}

static int check(const char *what, const double *x, int64_t n) {
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(x[i])) { fprintf(stderr, "%s[%lld] not finite\n", what, (long long)i); return 1; }
    return 0;
}

int main(void) {
    double h1[N * N], B[L * N * N];
    for (int p = 0; p < N; p++)
        for (int q = 0; q <= p; q++) h1[p * N + q] = h1[q * N + p] = (p == q) ? (p < NC ? -2.0 : p - 2.0) : 0.1 * urand();
    for (int l = 0; l < L; l++)
        for (int p = 0; p < N; p++)
            for (int q = 0; q <= p; q++) B[(l * N + p) * N + q] = B[(l * N + q) * N + p] = 0.2 * urand();
    orc_t *o = orc_create(N, NC, NA, NC + 1, NC + 1);
    if (!o) return 2;
    if (orc_set_integrals_chol(o, h1, B, L, 0.3)) return 3;
    /* reference: every active determinant with one active electron per spin,
     * as (alpha word, beta word), sorted with the beta word most significant
     * (the order the oracle requires) */
    uint64_t ref[NA * NA * 2];
    double c[NA * NA];
    int nr = 0;
    for (int b = 0; b < NA; b++)
        for (int a = 0; a < NA; a++) {
            ref[2 * nr] = 1ull | (1ull << (NC + a));
            ref[2 * nr + 1] = 1ull | (1ull << (NC + b));
            c[nr] = 0.5 + urand();
            nr++;
        }
    if (orc_set_reference(o, nr, ref, c)) return 4;
    int64_t ncls = orc_n_classes(o);
    double *cc = malloc(sizeof(double) * (size_t)(ncls - 1));
    for (int64_t i = 0; i < ncls - 1; i++) cc[i] = 0.1 + 0.05 * urand();
    if (orc_set_coeffs(o, 1.0, cc, ncls - 1)) return 5;
    double eps[N - NC - NA];
    for (int a = 0; a < N - NC - NA; a++) eps[a] = 1.0 + a;
    double e0 = orc_reference_energy(o);
    orc_set_dyall(o, eps, e0);
    orc_set_options(o, 0.0, 1);
    /* walkers: a reference determinant and first-order-space determinants */
    uint64_t w[4 * 2] = {ref[0], ref[1], 1ull | (1ull << 5), ref[3], 1ull | (1ull << 4), 1ull | (1ull << 6),
                         ref[8], 1ull | (1ull << 6)};
    int rc = 0;
    double el[4], ps[4], ga[4], ed[4], sa[4], ka[4];
    int64_t cl[4];
    orc_eval(o, 4, w, el, ps, ga, ed, cl, sa, ka, 2);
    rc |= check("psi", ps, 4) | check("gamma", ga, 4);
    for (int i = 0; i < 4; i++)
        if (ps[i] != 0.0) rc |= check("eloc", el + i, 1);
    int64_t nn = orc_neighbors(o, w, 0, NULL, NULL, NULL, NULL, NULL, NULL);
    uint64_t *nd = malloc(sizeof(uint64_t) * 2 * (size_t)nn);
    int8_t *ph = malloc((size_t)nn);
    double *hv = malloc(sizeof(double) * (size_t)nn), *pv = malloc(sizeof(double) * (size_t)nn),
           *hd = malloc(sizeof(double) * (size_t)nn);
    int64_t *nc = malloc(sizeof(int64_t) * (size_t)nn);
    orc_neighbors(o, w, nn, nd, ph, hv, pv, hd, nc);
    rc |= check("h", hv, nn) | check("psi(m)", pv, nn);
    double wsum[4 * 3] = {0}, *csum = calloc((size_t)ncls * 4, sizeof(double)), pout[4];
    uint64_t ww[8];
    memcpy(ww, w, sizeof(ww));
    int64_t stuck = orc_run(o, 2, ww, pout, 11, 0, 20, 5, 0, wsum, csum, 2);
    rc |= check("wsum", wsum, 6) | check("csum", csum, ncls * 4) | (stuck != 0);
    int64_t nnz = orc_det_hamiltonian(o, nr, ref, 0, NULL, NULL, NULL);
    int64_t *ri = malloc(sizeof(int64_t) * (size_t)nnz), *ci = malloc(sizeof(int64_t) * (size_t)nnz);
    double *hvv = malloc(sizeof(double) * (size_t)nnz);
    orc_det_hamiltonian(o, nr, ref, nnz, ri, ci, hvv);
    rc |= check("H", hvv, nnz);
    double g[NA * NA];
    orc_reference_rdm1(o, g);
    rc |= check("rdm1", g, NA * NA);
    int64_t tr[5];
    orc_traffic(o, w + 2, tr);
    rc |= (tr[3] != orc_neighbors(o, w + 2, 0, NULL, NULL, NULL, NULL, NULL, NULL));
    double p1 = orc_psi(o, w + 4);
    rc |= check("psi1", &p1, 1);
    free(cc); free(nd); free(ph); free(hv); free(pv); free(hd); free(nc); free(csum); free(ri); free(ci); free(hvv);
    orc_destroy(o);
    printf("oracle sanitizer run: %s (%lld neighbours, %lld Hamiltonian entries)\n", rc ? "FAILED" : "clean",
           (long long)nn, (long long)nnz);
    return rc;
}
