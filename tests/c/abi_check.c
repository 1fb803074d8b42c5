/*
 * abi_check.c -- the C ABI of libeofa.so used from plain C99 (no Python, no
 * torch): device memory through the HIP runtime API, a random SU(3) field,
 * and checks against the CPU oracle (test infrastructure, liboracle.so).
 *
 *   1. dwf_apply (D_DWF of eq. (2.3) and its adjoint, FP64) against the
 *      oracle's D_DWF, element by element;
 *   2. eofa_solve with the FP16 inner solver: the true residual reported,
 *      S against the oracle's action on the same chi (eq. (2.5)), and S
 *      against the oracle's own Cayley-form solve;
 *   3. the gauge action and force (zero on unit links), the dense D_EOFA
 *      solve (same action), the force (finite), the MD update (kinetic
 *      term), and the heatbath on a Lanczos interval (phi^dag M phi =
 *      eta^dag eta within the approximation error);
 *   4. error paths: m1 > m2 and a NULL context give EOFA_EINVAL with a message.
 *
 * Prints "abi_check: ok" and exits 0, or names the failed check and exits 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "eofa.h"

/* oracle entry points (oracle/oracle.c) */
typedef struct {
    int L[4];
    int Ls;
    int antiperiodic_t;
    double M5;
    double b5, c5;
} og_t;
void orc_ddwf(const og_t *g, const double *U, double mp, double mm, int dagger, const double *in,
              double *out);
int orc_eofa_chi(const og_t *g, const double *U, double m1, double m2, const double *phi, double *chiL,
                 double *chiR, int method, double tol, int maxiter, int *iters);
void orc_action(const og_t *g, double m1, double m2, const double *phi, const double *chiL,
                const double *chiR, double *S, double *Mphi);

static int failures = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            fprintf(stderr, "abi_check: FAILED: " __VA_ARGS__); \
            fprintf(stderr, "\n");                        \
            ++failures;                                   \
        }                                                 \
    } while (0)

/* xorshift64* -> uniform in [-1, 1) */
static uint64_t rs = 0x9e3779b97f4a7c15ull;
static double urand(void) {
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return (double)((rs * 0x2545f4914f6cdd1dull) >> 11) / 4503599627370496.0 - 1.0;
}

/* random SU(3): orthonormalise two random complex rows, third = conj(r0 x r1) */
static void random_su3(double *m) {
    double a[2][6];
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 6; ++q) a[r][q] = urand();
    double n0 = 0;
    for (int q = 0; q < 6; ++q) n0 += a[0][q] * a[0][q];
    n0 = sqrt(n0);
    for (int q = 0; q < 6; ++q) a[0][q] /= n0;
    double dr = 0, di = 0;   /* <r0, r1> = sum conj(r0) r1 */
    for (int c = 0; c < 3; ++c) {
        dr += a[0][2 * c] * a[1][2 * c] + a[0][2 * c + 1] * a[1][2 * c + 1];
        di += a[0][2 * c] * a[1][2 * c + 1] - a[0][2 * c + 1] * a[1][2 * c];
    }
    for (int c = 0; c < 3; ++c) {
        a[1][2 * c] -= dr * a[0][2 * c] - di * a[0][2 * c + 1];
        a[1][2 * c + 1] -= dr * a[0][2 * c + 1] + di * a[0][2 * c];
    }
    double n1 = 0;
    for (int q = 0; q < 6; ++q) n1 += a[1][q] * a[1][q];
    n1 = sqrt(n1);
    for (int q = 0; q < 6; ++q) a[1][q] /= n1;
    memcpy(m, a[0], 6 * sizeof(double));
    memcpy(m + 6, a[1], 6 * sizeof(double));
    for (int c = 0; c < 3; ++c) {   /* (r0 x r1)_c conjugated */
        const int i = (c + 1) % 3, j = (c + 2) % 3;
        const double xr = a[0][2 * i] * a[1][2 * j] - a[0][2 * i + 1] * a[1][2 * j + 1]
                        - (a[0][2 * j] * a[1][2 * i] - a[0][2 * j + 1] * a[1][2 * i + 1]);
        const double xi = a[0][2 * i] * a[1][2 * j + 1] + a[0][2 * i + 1] * a[1][2 * j]
                        - (a[0][2 * j] * a[1][2 * i + 1] + a[0][2 * j + 1] * a[1][2 * i]);
        m[12 + 2 * c] = xr;
        m[12 + 2 * c + 1] = -xi;
    }
}

static double rel_diff(const double *a, const double *b, size_t n) {
    double d = 0, r = 0;
    for (size_t i = 0; i < n; ++i) {
        d += (a[i] - b[i]) * (a[i] - b[i]);
        r += b[i] * b[i];
    }
    return sqrt(d / r);
}

static void *dev_copy(const double *h, size_t n) {
    void *d = NULL;
    if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) return NULL;
    if (h && hipMemcpy(d, h, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return NULL;
    return d;
}

int main(void) {
    const eofa_geom_t geom = {{4, 4, 4, 4}, 8, 1.8, 2.0, 1};
    const int V = 256, Ls = 8;
    const og_t og = {{4, 4, 4, 4}, 8, 1, 1.8, 1.5, 0.5};   /* b5 = (alpha+1)/2, c5 = (alpha-1)/2 */
    const size_t nU = (size_t)4 * V * 18, n5 = (size_t)Ls * V * 24, n4 = (size_t)V * 24;
    double *U = malloc(nU * sizeof(double)), *psi = malloc(n5 * sizeof(double));
    double *out = malloc(n5 * sizeof(double)), *ref = malloc(n5 * sizeof(double));
    double *phi = malloc(n4 * sizeof(double));
    double *chiL = malloc(n5 * sizeof(double)), *chiR = malloc(n5 * sizeof(double));
    double *rL = malloc(n5 * sizeof(double)), *rR = malloc(n5 * sizeof(double));
    for (size_t l = 0; l < (size_t)4 * V; ++l) random_su3(U + 18 * l);
    for (size_t i = 0; i < n5; ++i) psi[i] = urand();
    for (size_t i = 0; i < n4; ++i) phi[i] = urand();

    void *dU = dev_copy(U, nU), *dpsi = dev_copy(psi, n5), *dout = dev_copy(NULL, n5);
    void *dphi = dev_copy(phi, n4), *dchiL = dev_copy(NULL, n5), *dchiR = dev_copy(NULL, n5);
    if (!dU || !dpsi || !dout || !dphi || !dchiL || !dchiR) {
        fprintf(stderr, "abi_check: FAILED: device allocation\n");
        return 1;
    }
    eofa_ctx_t *ctx = NULL;
    int rc = eofa_ctx_create(&ctx, &geom, dU, NULL);
    CHECK(rc == EOFA_OK && ctx, "eofa_ctx_create: %d %s", rc, eofa_last_error());
    if (!ctx) return 1;

    /* 1. D_DWF and its adjoint against the oracle */
    for (int dag = 0; dag < 2; ++dag) {
        rc = dwf_apply(ctx, 0.04, 0.7, dag, 0, EOFA_FP64, dpsi, dout);
        CHECK(rc == EOFA_OK, "dwf_apply: %d %s", rc, eofa_last_error());
        hipMemcpy(out, dout, n5 * sizeof(double), hipMemcpyDeviceToHost);
        orc_ddwf(&og, U, 0.04, 0.7, dag, psi, ref);
        const double r = rel_diff(out, ref, n5);
        CHECK(r < 1e-13, "dwf_apply(dagger=%d) differs from the oracle: %.3e", dag, r);
    }

    /* 2. EOFA solves with the FP16 inner solver, and the action */
    const double m1 = 0.04, m2 = 1.0;
    eofa_solver_t sp = {1e-10, 20000, EOFA_FP16, 0.3, 0};
    eofa_stats_t st;
    double S = 0;
    rc = eofa_solve(ctx, m1, m2, dphi, NULL, NULL, dchiL, dchiR, NULL, &S, &sp, &st);
    CHECK(rc == EOFA_OK, "eofa_solve: %d %s", rc, eofa_last_error());
    CHECK(st.true_resid[0] <= 1e-10 && st.true_resid[1] <= 1e-10, "true residual %.3e %.3e",
          st.true_resid[0], st.true_resid[1]);
    CHECK(st.inner_used[0] == EOFA_FP16 && st.inner_used[1] == EOFA_FP16, "inner precision escalated");
    hipMemcpy(chiL, dchiL, n5 * sizeof(double), hipMemcpyDeviceToHost);
    hipMemcpy(chiR, dchiR, n5 * sizeof(double), hipMemcpyDeviceToHost);
    double S2[2];
    orc_action(&og, m1, m2, phi, chiL, chiR, S2, NULL);
    CHECK(fabs(S - S2[0]) <= 1e-13 * fabs(S2[0]), "action kernel: %.15e vs oracle %.15e", S, S2[0]);
    int its[2];
    rc = orc_eofa_chi(&og, U, m1, m2, phi, rL, rR, 1, 1e-13, 100000, its);
    CHECK(rc == 0, "oracle solve did not converge");
    orc_action(&og, m1, m2, phi, rL, rR, S2, NULL);
    CHECK(fabs(S - S2[0]) <= 1e-9 * fabs(S2[0]), "S = %.15e, oracle %.15e", S, S2[0]);

    /* 3. the other entry points, each with a property that fixes its answer */
    {
        /* gauge action and force of unit links: exactly zero */
        double *one = calloc(nU, sizeof(double));
        for (size_t l = 0; l < (size_t)4 * V; ++l)
            for (int a = 0; a < 3; ++a) one[18 * l + 8 * a] = 1.0;
        void *done = dev_copy(one, nU), *dF = dev_copy(NULL, nU);
        double Sg = -1;
        rc = eofa_gauge_action(ctx, done, 2.13, -0.331, &Sg);
        CHECK(rc == EOFA_OK && Sg == 0.0, "gauge action of unit links: %d %g", rc, Sg);
        rc = eofa_gauge_force(ctx, done, 2.13, -0.331, dF, 0);
        hipMemcpy(one, dF, nU * sizeof(double), hipMemcpyDeviceToHost);
        double fbig = 0;
        for (size_t i = 0; i < nU; ++i) fbig = fbig > fabs(one[i]) ? fbig : fabs(one[i]);
        CHECK(rc == EOFA_OK && fbig == 0.0, "gauge force of unit links: %d %g", rc, fbig);
        rc = eofa_gauge_action(ctx, dU, 2.13, -0.331, &Sg);
        CHECK(rc == EOFA_OK && Sg > 0.0 && isfinite(Sg), "gauge action of random links: %d %g", rc, Sg);

        /* the dense D_EOFA path (FP32 inner) solves the same systems */
        eofa_solver_t sp32 = {1e-10, 20000, EOFA_FP32, 0.3, 0};
        double Sd = 0;
        rc = eofa_solve_dense(ctx, m1, m2, dphi, dchiL, dchiR, NULL, &Sd, &sp32, &st);
        CHECK(rc == EOFA_OK && fabs(Sd - S) <= 1e-9 * fabs(S), "dense solve: %d %.15e vs %.15e", rc, Sd, S);

        /* the force from those solutions is finite */
        rc = eofa_force(ctx, m1, m2, dphi, dchiL, dchiR, dF, NULL, &sp, NULL);
        hipMemcpy(one, dF, nU * sizeof(double), hipMemcpyDeviceToHost);
        int fin = 1;
        for (size_t i = 0; i < nU; ++i) fin = fin && isfinite(one[i]);
        CHECK(rc == EOFA_OK && fin, "force: %d", rc);

        /* MD update with dt = 0: only the kinetic term, P and U untouched */
        double *P = calloc(nU, sizeof(double)), kin = -1;
        for (size_t l = 0; l < (size_t)4 * V; ++l) { P[18 * l] = 0.5; P[18 * l + 8] = -0.5; }   /* diag(1/2, -1/2, 0) */
        void *dP = dev_copy(P, nU);
        rc = eofa_md_update(ctx, dU, dP, NULL, 0.0, 0.0, &kin);
        CHECK(rc == EOFA_OK && fabs(kin - 0.5 * 4 * V) <= 1e-12 * V, "md kinetic: %d %g", rc, kin);

        /* heatbath of eq. (3.1): phi^dag M_EOFA phi = eta^dag eta up to the
         * approximation error on an interval from the Lanczos bounds */
        double th[2], res[2];
        eofa_solver_t spb = {1e-8, 20000, EOFA_FP64, 0.3, 1};
        rc = eofa_meofa_bounds(ctx, m1, m2, dphi, 20, &spb, th, res, NULL);
        CHECK(rc == EOFA_OK && th[0] > 0 && th[1] > th[0], "meofa bounds: %d %g %g", rc, th[0], th[1]);
        double a0, al[8], be[8], delta;
        const double lo = 0.9 * fmax(th[0] - res[0], 0.5 * th[0]), hi = 1.1 * (th[1] + res[1]);
        rc = eofa_rational_inv_sqrt(lo, hi, 6, &a0, al, be, &delta);
        CHECK(rc == EOFA_OK, "rational coefficients: %d", rc);
        void *deta = dev_copy(phi, n4), *dphi2 = dev_copy(NULL, n4);
        rc = eofa_heatbath(ctx, m1, m2, deta, 6, a0, al, be, 4, dphi2, &sp, &st);
        CHECK(rc == EOFA_OK, "heatbath: %d %s", rc, eofa_last_error());
        double Sh = 0, ee = 0;
        rc = eofa_solve(ctx, m1, m2, dphi2, NULL, NULL, dchiL, dchiR, NULL, &Sh, &sp, &st);
        for (size_t i = 0; i < n4; ++i) ee += phi[i] * phi[i];
        CHECK(rc == EOFA_OK && fabs(Sh / ee - 1.0) <= 2.01 * delta + 1e-8,
              "heatbath: S/eta^2 - 1 = %.3e, delta %.3e", Sh / ee - 1.0, delta);
        hipFree(done); hipFree(dF); hipFree(dP); hipFree(deta); hipFree(dphi2);
        free(one); free(P);
    }

    /* 4. error paths */
    rc = eofa_solve(ctx, m2, m1, dphi, NULL, NULL, dchiL, dchiR, NULL, &S, &sp, &st);
    CHECK(rc == EOFA_EINVAL && strlen(eofa_last_error()) > 0, "m1 > m2 not rejected: %d", rc);
    CHECK(dwf_apply(NULL, 0.1, 0.1, 0, 0, EOFA_FP64, dpsi, dout) == EOFA_EINVAL, "NULL context not rejected");

    eofa_ctx_destroy(ctx);
    hipFree(dU); hipFree(dpsi); hipFree(dout); hipFree(dphi); hipFree(dchiL); hipFree(dchiR);
    free(U); free(psi); free(out); free(ref); free(phi); free(chiL); free(chiR); free(rL); free(rR);
    if (failures) return 1;
    printf("abi_check: ok (S = %.12e, iterations %d + %d)\n", S, st.iters[0], st.iters[1]);
    return 0;
}
