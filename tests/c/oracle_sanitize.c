/*
 * oracle_sanitize.c -- every entry point of the C oracle (oracle/oracle.c)
 * on a tiny lattice with an odd Ls, for an AddressSanitizer and
 * UndefinedBehaviorSanitizer build of the oracle's sources.  It checks only
 * that each call runs clean and returns finite numbers; the oracle's values
 * are pinned by the Python tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int L[4];
    int Ls;
    int antiperiodic_t;
    double M5;
    double b5, c5;
} og_t;

void orc_gamma(int mu, double *out);
void orc_wilson(const og_t *g, const double *U, const double *in, double *out, int nslice, int dagger);
void orc_L(const og_t *g, double mp, double mm, int transpose, const double *in, double *out);
int orc_chiral_matrix(const og_t *g, int which, int plus, double m, double *A);
int orc_apply_chiral(const og_t *g, int which, double mp, double mm, int transpose, const double *in,
                     double *out);
void orc_ddwf(const og_t *g, const double *U, double mp, double mm, int dagger, const double *in,
              double *out);
void orc_deofa(const og_t *g, const double *U, double mp, double mm, const double *in, double *out);
void orc_g5r5(const og_t *g, const double *in, double *out);
void orc_H(const og_t *g, const double *U, double mp, double mm, const double *in, double *out);
void orc_omega_k(const og_t *g, double m1, double m2, double *om_minus, double *om_plus, double *k);
void orc_schur(const og_t *g, const double *U, double mp, double mm, int dagger, const double *in,
               double *out);
int orc_solve_ddwf_eo(const og_t *g, const double *U, double mp, double mm, const double *b, double *y,
                      double tol, int maxiter, int fixed, double *resid);
int orc_solve_H(const og_t *g, const double *U, double mp, double mm, const double *v, double *chi,
                double tol, int maxiter, double *resid);
void orc_H_shifted(const og_t *g, const double *U, double m1, double m2, int which, double gshift,
                   const double *in, double *out);
int orc_solve_H_shifted(const og_t *g, const double *U, double m1, double m2, int which, double gshift,
                        const double *v, double *chi, double tol, int maxiter, double *resid);
int orc_eofa_chi(const og_t *g, const double *U, double m1, double m2, const double *phi, double *chiL,
                 double *chiR, int method, double tol, int maxiter, int *iters);
void orc_action(const og_t *g, double m1, double m2, const double *phi, const double *chiL,
                const double *chiR, double *S, double *Mphi);
void orc_force(const og_t *g, const double *U, double m1, double m2, const double *chiL,
               const double *chiR, double *F, double *G, const int *links, long nlinks);
void orc_ddwf_sites(const og_t *g, const double *U, double mp, double mm, int dagger, const double *in,
                    const long *sites, long n, double *out);
void orc_schur_sites(const og_t *g, const double *U, double mp, double mm, int dagger, const double *in,
                     const long *sites, long n, double *out);

static uint64_t rs = 0x853c49e6748fea9bull;
static double urand(void) {
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return (double)((rs * 0x2545f4914f6cdd1dull) >> 11) / 4503599627370496.0 - 1.0;
}

/* unitary 3x3 by Gram-Schmidt of random complex rows (det not fixed: the
 * oracle needs no SU(3) here, only finite links) */
static void random_u3(double *m) {
    double a[3][6];
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 6; ++q) a[r][q] = urand();
        for (int p = 0; p < r; ++p) {
            double dr = 0, di = 0;
            for (int c = 0; c < 3; ++c) {
                dr += a[p][2 * c] * a[r][2 * c] + a[p][2 * c + 1] * a[r][2 * c + 1];
                di += a[p][2 * c] * a[r][2 * c + 1] - a[p][2 * c + 1] * a[r][2 * c];
            }
            for (int c = 0; c < 3; ++c) {
                a[r][2 * c] -= dr * a[p][2 * c] - di * a[p][2 * c + 1];
                a[r][2 * c + 1] -= dr * a[p][2 * c + 1] + di * a[p][2 * c];
            }
        }
        double n = 0;
        for (int q = 0; q < 6; ++q) n += a[r][q] * a[r][q];
        n = sqrt(n);
        for (int q = 0; q < 6; ++q) a[r][q] /= n;
    }
    memcpy(m, a, sizeof(a));
}

static int bad = 0;
static void finite(const char *what, const double *x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) {
            fprintf(stderr, "oracle_sanitize: %s is not finite\n", what);
            ++bad;
            return;
        }
}

int main(void) {
    const og_t g = {{2, 2, 2, 4}, 3, 1, 1.8, 1.5, 0.5};
    const long V = 32, Ls = 3;
    const size_t nU = (size_t)4 * V * 18, n5 = (size_t)Ls * V * 24, n4 = (size_t)V * 24;
    double *U = malloc(nU * 8), *a = malloc(n5 * 8), *b = malloc(n5 * 8), *c = malloc(n5 * 8);
    double *phi = malloc(n4 * 8), *F = malloc(nU * 8), *G = malloc(nU * 8), *M = malloc(n4 * 8);
    double gam[32], A[9], omm[3], omp[3], k, S[2], res;
    for (size_t l = 0; l < (size_t)4 * V; ++l) random_u3(U + 18 * l);
    for (size_t i = 0; i < n5; ++i) a[i] = urand();
    for (size_t i = 0; i < n4; ++i) phi[i] = urand();

    for (int mu = 0; mu < 5; ++mu) orc_gamma(mu, gam);
    finite("gamma", gam, 32);
    for (int dag = 0; dag < 2; ++dag) {
        orc_wilson(&g, U, a, b, (int)Ls, dag);
        finite("wilson", b, n5);
        orc_wilson(&g, U, a, b, 1, dag);
        orc_L(&g, 0.1, 0.3, dag, a, b);
        finite("L", b, n5);
        orc_ddwf(&g, U, 0.1, 0.3, dag, a, b);
        finite("ddwf", b, n5);
        orc_schur(&g, U, 0.1, 0.3, dag, a, b);
        finite("schur", b, n5);
    }
    for (int which = 0; which < 6; ++which)
        for (int plus = 0; plus < 2; ++plus) {
            if (orc_chiral_matrix(&g, which, plus, 0.2, A)) ++bad;
            finite("chiral matrix", A, 9);
            if (orc_apply_chiral(&g, which, 0.1, 0.3, plus, a, b)) ++bad;
            finite("apply chiral", b, n5);
        }
    orc_deofa(&g, U, 0.1, 0.3, a, b);
    finite("deofa", b, n5);
    orc_g5r5(&g, a, b);
    orc_H(&g, U, 0.1, 0.3, a, b);
    finite("H", b, n5);
    orc_omega_k(&g, 0.1, 0.6, omm, omp, &k);
    finite("omega", omm, 3);
    if (orc_solve_ddwf_eo(&g, U, 0.1, 0.3, a, b, 1e-10, 5000, 0, &res) >= 5000) ++bad;
    orc_solve_ddwf_eo(&g, U, 0.1, 0.3, a, b, 1e-10, 5000, 7, &res);
    finite("solve_ddwf_eo", b, n5);
    if (orc_solve_H(&g, U, 0.1, 0.3, a, b, 1e-10, 5000, &res) >= 5000) ++bad;
    for (int which = 0; which < 2; ++which) {
        orc_H_shifted(&g, U, 0.1, 0.6, which, 0.4, a, b);
        finite("H shifted", b, n5);
        if (orc_solve_H_shifted(&g, U, 0.1, 0.6, which, 0.4, a, b, 1e-10, 5000, &res) >= 5000) ++bad;
    }
    int its[2];
    for (int method = 0; method < 2; ++method)
        if (orc_eofa_chi(&g, U, 0.1, 0.6, phi, b, c, method, 1e-10, 5000, its)) ++bad;
    orc_action(&g, 0.1, 0.6, phi, b, c, S, M);
    finite("action", S, 2);
    finite("M_EOFA phi", M, n4);
    orc_force(&g, U, 0.1, 0.6, b, c, F, G, NULL, 0);
    finite("force", F, nU);
    finite("gradient", G, nU);
    const int links[6] = {0, 0, 3, 31, 1, 17};
    orc_force(&g, U, 0.1, 0.6, b, c, F, G, links, 3);
    finite("force at links", F, 3 * 18);
    const long sites[6] = {0, 0, 2, 31, 1, 1};   /* (s, natural site) */
    orc_ddwf_sites(&g, U, 0.1, 0.3, 0, a, sites, 3, b);
    finite("ddwf sites", b, 3 * 24);
    const long odd[4] = {0, 1, 2, 30};   /* (s, odd natural site): x+y+z+t = 1 and 5 */
    orc_schur_sites(&g, U, 0.1, 0.3, 1, a, odd, 2, b);
    finite("schur sites", b, 2 * 24);

    free(U); free(a); free(b); free(c); free(phi); free(F); free(G); free(M);
    if (bad) return 1;
    printf("oracle_sanitize: ok\n");
    return 0;
}
