/*
 * host_sanitize.c -- the host-side paths of the C ABI, for a build of
 * libeofa.so whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (device code unchanged):
 *   - Zolotarev coefficients (eofa_rational_inv_sqrt), valid and invalid;
 *   - argument validation of every entry point with a NULL context;
 *   - context creation rejecting bad geometry, and, where the HIP runtime
 *     sees no device at all, failing at its first device call and
 *     releasing what it had set up.
 * Prints "host_sanitize: ok" and exits 0, or names the failure and exits 1.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "eofa.h"

static int bad = 0;
#define EXPECT(cond, what)                                        \
    do {                                                          \
        if (!(cond)) {                                            \
            fprintf(stderr, "host_sanitize: FAILED: %s\n", what); \
            ++bad;                                                \
        }                                                         \
    } while (0)

int main(void) {
    double a0, al[64], be[64], delta;
    const double iv[][2] = {{0.5, 5.0}, {0.9, 27.9}, {1e-3, 1e3}, {2.0, 2.0}};
    for (int k = 0; k < 4; ++k)
        for (int n = 1; n <= 32; n *= 2) {
            const int rc = eofa_rational_inv_sqrt(iv[k][0], iv[k][1], n, &a0, al, be, &delta);
            EXPECT(rc == EOFA_OK, "rational coefficients");
            int finite = isfinite(a0) && isfinite(delta);
            for (int l = 0; l < n; ++l) finite = finite && isfinite(al[l]) && isfinite(be[l]);
            EXPECT(finite, "non-finite coefficient");
        }
    EXPECT(eofa_rational_inv_sqrt(-1.0, 2.0, 4, &a0, al, be, &delta) == EOFA_EINVAL, "lo < 0 accepted");
    EXPECT(eofa_rational_inv_sqrt(3.0, 2.0, 4, &a0, al, be, &delta) == EOFA_EINVAL, "lo > hi accepted");
    EXPECT(eofa_rational_inv_sqrt(1.0, 2.0, 0, &a0, al, be, &delta) == EOFA_EINVAL, "n = 0 accepted");
    EXPECT(eofa_rational_inv_sqrt(1.0, 2.0, 4, NULL, al, be, &delta) == EOFA_EINVAL, "NULL accepted");
    EXPECT(strlen(eofa_last_error()) > 0, "no error message");

    const eofa_solver_t sp = {1e-10, 100, EOFA_FP64, 0.3, 0};
    eofa_stats_t st;
    double S, th[2], r[2];
    EXPECT(dwf_apply(NULL, 0.1, 0.1, 0, 0, EOFA_FP64, NULL, NULL) == EOFA_EINVAL, "dwf_apply");
    EXPECT(eofa_solve(NULL, 0.1, 0.2, NULL, NULL, NULL, NULL, NULL, NULL, &S, &sp, &st) == EOFA_EINVAL,
           "eofa_solve");
    EXPECT(eofa_solve_dense(NULL, 0.1, 0.2, NULL, NULL, NULL, NULL, &S, &sp, &st) == EOFA_EINVAL,
           "eofa_solve_dense");
    EXPECT(eofa_force(NULL, 0.1, 0.2, NULL, NULL, NULL, NULL, NULL, &sp, &st) == EOFA_EINVAL, "eofa_force");
    EXPECT(eofa_md_update(NULL, NULL, NULL, NULL, 0.1, 0.1, NULL) == EOFA_EINVAL, "eofa_md_update");
    EXPECT(eofa_heatbath(NULL, 0.1, 0.2, NULL, 1, 1.0, al, be, 0, NULL, &sp, &st) == EOFA_EINVAL,
           "eofa_heatbath");
    EXPECT(eofa_meofa_bounds(NULL, 0.1, 0.2, NULL, 8, &sp, th, r, &st) == EOFA_EINVAL, "eofa_meofa_bounds");
    EXPECT(eofa_chrono(NULL, 4) == EOFA_EINVAL, "eofa_chrono");
    EXPECT(eofa_gauge_action(NULL, NULL, 2.0, -0.331, &S) == EOFA_EINVAL, "eofa_gauge_action");
    EXPECT(eofa_gauge_force(NULL, NULL, 2.0, -0.331, NULL, 0) == EOFA_EINVAL, "eofa_gauge_force");
    EXPECT(eofa_ctx_update_gauge(NULL, NULL) == EOFA_EINVAL, "eofa_ctx_update_gauge");
    EXPECT(eofa_timing_enable(NULL, 1) == EOFA_EINVAL, "eofa_timing_enable");
    eofa_ctx_destroy(NULL);

    eofa_ctx_t *ctx = NULL;
    const eofa_geom_t odd = {{3, 4, 4, 4}, 8, 1.8, 2.0, 1}, ls0 = {{4, 4, 4, 4}, 0, 1.8, 2.0, 1};
    EXPECT(eofa_ctx_create(&ctx, &odd, (const void *)&odd, NULL) == EOFA_EINVAL && !ctx, "odd extent");
    EXPECT(eofa_ctx_create(&ctx, &ls0, (const void *)&odd, NULL) == EOFA_EINVAL && !ctx, "Ls = 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (ndev == 0) {   /* no device: creation must fail cleanly at its first device call */
        const eofa_geom_t good = {{4, 4, 4, 4}, 8, 1.8, 2.0, 1};
        const int rc = eofa_ctx_create(&ctx, &good, (const void *)&good, NULL);
        EXPECT(rc != EOFA_OK && !ctx, "context created without a device");
    }
    if (bad) return 1;
    printf("host_sanitize: ok (%d device(s))\n", ndev);
    return 0;
}
