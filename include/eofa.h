/*
 * eofa.h -- C ABI of the MI355X (gfx950) EOFA hot-path library.
 *
 * Exact one-flavour algorithm for Moebius domain wall fermions, after
 * D. Murphy, "Domain Wall Fermion Simulations with the Exact One-Flavor
 * Algorithm", LATTICE 2016 (arXiv:1611.00298).
 *
 * Conventions (the paper leaves them open; every entry point uses these):
 *   - lattice L = (Lx, Ly, Lz, Lt), every extent even; 4D site index
 *     i = x + Lx*(y + Ly*(z + Lz*t)); V = Lx*Ly*Lz*Lt; s = 0..Ls-1.
 *   - chiral gamma basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *     gamma_t = [[0,1],[1,0]], gamma_5 = diag(1,1,-1,-1); P+ = spins {0,1}.
 *   - D_w psi(x) = (4-M5) psi(x) - 1/2 sum_mu [(1-gamma_mu) U_mu(x) psi(x+mu)
 *       + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu)], periodic in space and
 *     (optionally) antiperiodic in t.
 *   - L = P+ L+(m+) + P- L-(m-): (L+ v)_s = v_{s-1}, (L+ v)_0 = -m+ v_{Ls-1};
 *     (L- v)_s = v_{s+1}, (L- v)_{Ls-1} = -m- v_0.
 *   - b5 = (alpha+1)/2 and c5 = (alpha-1)/2 are the paper's c+d and c-d
 *     (Section 2: c = alpha/2, d = 1/2).
 *   - D_DWF(m+, m-) = D_w (b5 + c5 L) + (1 - L)            (eq. (2.3))
 *   - Dtilde = b5 + c5 L; D_EOFA = D_DWF Dtilde^-1;
 *     H(m+, m-) = gamma_5 R_5 D_EOFA(m+, m-)               (Section 2)
 *
 * Memory: every pointer named *_dev is a device pointer on the GPU that is
 * current when the context is created, C-contiguous complex128 (pairs of
 * doubles, real first), owned by the caller.  The library never frees or
 * keeps a caller pointer beyond the call.  Layouts (natural):
 *   gauge  U[mu][t][z][y][x][a][b]            4*V*9 complex
 *   4D     phi[t][z][y][x][spin][colour]      V*12 complex
 *   5D     psi[s][t][z][y][x][spin][colour]   Ls*V*12 complex
 * All work is enqueued on the stream given at context creation; calls
 * that return scalars (S, kinetic energy, statistics) synchronise it.
 *
 * Errors: every int-returning call gives EOFA_OK (0) or a negative code;
 * eofa_last_error() then holds a message for the calling thread.  No C++
 * exception crosses this interface.
 */
#ifndef EOFA_H
#define EOFA_H

#ifdef __cplusplus
extern "C" {
#endif

#define EOFA_OK       0
#define EOFA_EINVAL  -1   /* bad argument: odd extent, Ls out of range, NULL, m1 > m2, N(m) <= 0 */
#define EOFA_ENOMEM  -2   /* device allocation failed */
#define EOFA_ENOCONV -3   /* solver hit maxiter; outputs and statistics are still written */
#define EOFA_ENAN    -4   /* a reduction produced NaN or Inf */
#define EOFA_EDEVICE -5   /* a HIP runtime call failed */

typedef struct eofa_ctx eofa_ctx_t;

typedef enum {
    EOFA_FP64 = 0,   /* double everywhere */
    EOFA_FP32 = 1,   /* float storage and arithmetic */
    EOFA_FP16 = 2,   /* IEEE half storage with one float norm per 5D site, float arithmetic */
    EOFA_BF16 = 3    /* bfloat16 storage, float arithmetic */
} eofa_prec_t;

typedef struct {
    int L[4];            /* Lx, Ly, Lz, Lt; each even and >= 2 */
    int Ls;              /* extent of the fifth dimension, 1 <= Ls <= 64 */
    double M5;           /* domain-wall height (Wilson mass -M5) */
    double alpha;        /* Moebius scale (Section 2); alpha = 1 is Shamir */
    int antiperiodic_t;  /* 1: antiperiodic in t, 0: periodic */
} eofa_geom_t;

typedef struct {
    double tol;            /* target true residual |b - D_DWF y| / |b| per system */
    int maxiter;           /* limit on inner CG iterations per system */
    eofa_prec_t inner;     /* EOFA_FP64: plain CGNR; else reliable-update mixed precision */
    double reliable_delta; /* reliable update when |r| falls below delta * |r| at the last update */
    int fused_fp64;        /* inner == EOFA_FP64 only (ignored otherwise).  0: plain CGNR, which
                              updates r, recomputes z = Mhat^dag r and reads |r|^2 on the host
                              every iteration.  1: the iteration of the mixed-precision solver run
                              entirely in FP64: z follows its own recursion inside the last hop
                              launch, the directions are kept as Dtilde p, the host reads the
                              scalars one iteration late, and FP64 reliable updates (every
                              reliable_delta of residual reduction) recompute the true residual.
                              It isolates the gain of the 16-bit and FP32 inner arithmetic from
                              that of these fusions.  eofa_solve, eofa_force, eofa_heatbath and
                              eofa_meofa_bounds honour it; eofa_solve_dense ignores it. */
} eofa_solver_t;

typedef struct {
    int iters[2];            /* CG iterations for (chi_L, chi_R) */
    int reliable_updates[2]; /* FP64 residual recomputations (mixed precision) */
    double true_resid[2];    /* |b - D_DWF y| / |b| recomputed in FP64 at the end */
    double seconds;          /* wall time of the call */
    double flops;            /* operator flops executed (1320 per Wilson hop per 5D site,
                                72 per bidiagonal 5D op, 144 per inverse 5D op) */
    eofa_prec_t inner_used[2]; /* the most precise inner arithmetic each system needed: the
                                  requested one, unless a 16-bit (then FP32) solve stopped
                                  making progress and continued one precision up (FP16/BF16
                                  -> FP32 -> FP64) from its current iterate */
} eofa_stats_t;

/* Create a context for one lattice geometry and gauge field.
 * U_dev: gauge field, natural layout (see above); copied and converted.
 * stream: hipStream_t (NULL for the default stream); all work goes there.
 * Returns EOFA_EINVAL for bad geometry, EOFA_ENOMEM, EOFA_EDEVICE. */
int eofa_ctx_create(eofa_ctx_t **ctx, const eofa_geom_t *geom, const void *U_dev, void *stream);

/* Free the context and every workspace it owns. NULL is allowed. */
void eofa_ctx_destroy(eofa_ctx_t *ctx);

/* Replace the gauge field (e.g. after a molecular-dynamics link update). */
int eofa_ctx_update_gauge(eofa_ctx_t *ctx, const void *U_dev);

/* Apply the Moebius domain-wall operator of eq. (2.3).
 *   eo = 0: out = D_DWF(m+, m-) in  (dagger: D_DWF^dag), full 5D fields.
 *   eo = 1: out = Mhat in on odd sites, the even-odd Schur complement
 *           Mhat = M_oo - M_oe M_ee^-1 M_eo of Section 5.1 (dagger: Mhat^dag);
 *           even sites of in are ignored and even sites of out are zero.
 * prec: arithmetic/storage precision of the operator (input and output
 * stay complex128).  in_dev/out_dev: 5D natural layout, may not alias. */
int dwf_apply(eofa_ctx_t *ctx, double m_plus, double m_minus, int dagger, int eo,
              eofa_prec_t prec, const void *in_dev, void *out_dev);

/* EOFA solves, action and M_EOFA phi (eqs. (2.5), (3.2), (5.1)).
 *   chi_L = H(m1, m1)^-1 Omega_- P_- phi,  chi_R = H(m1, m2)^-1 Omega_+ P_+ phi
 * (H(m2) - Delta_+ P_+ = H(m+ = m1, m- = m2)), computed in the Cayley form
 * chi = Dtilde D_DWF^-1 gamma_5 R_5 v (footnote of Section 5.1) with
 * even-odd CGNR.  Omega_-(s) = (-c5/b5)^s, Omega_+ = R_5 Omega_-,
 * k = (b5+c5) b5^(2Ls-2) (m2-m1) / (N(m1) N(m2)), N(m) = b5^Ls + m (-c5)^Ls.
 *   phi_dev: 4D pseudofermion.  x0_L/x0_R: initial guesses for chi (NULL: 0).
 *   chiL_dev/chiR_dev: 5D outputs.  Mphi_dev: 4D output M_EOFA phi (NULL: skip).
 *   S_out: S = phi^dag M_EOFA phi (NULL: skip).  stats may be NULL.
 * Requires m1 <= m2.  EOFA_ENOCONV leaves the best iterate in chi. */
int eofa_solve(eofa_ctx_t *ctx, double m1, double m2, const void *phi_dev,
               const void *x0_L_dev, const void *x0_R_dev, void *chiL_dev, void *chiR_dev,
               void *Mphi_dev, double *S_out, const eofa_solver_t *solver, eofa_stats_t *stats);

/* The same EOFA solves without the Cayley-form right preconditioning: the
 * comparison path of Table 4 ("EOFA (dense)").  Each system is solved as
 * D_EOFA chi = gamma_5 R_5 v with D_EOFA = D_w + (1 - L) Dtilde^-1, whose
 * 5D structure is dense: even-odd CGNR on
 *   Mhat = D5 - Dh_oe D5^-1 Dh_eo,  D5 = (4 - M5) + (1 - L) Dtilde^-1,
 * D5 applied as one Ls x Ls block per chirality.  The residual
 * b - D_EOFA chi equals the Cayley form's b - D_DWF y (chi = Dtilde y), so
 * `solver->tol` means the same in both.  solver->inner: EOFA_FP64 (plain
 * CGNR), EOFA_FP32 or EOFA_FP16 (that storage with FP32 arithmetic and FP64
 * reliable updates, as in eofa_solve); EOFA_BF16 gives EOFA_EINVAL.  No
 * initial guesses.  A 16-bit (then FP32) inner solve that stops making
 * progress (no halving of the true residual in 1000 iterations, or a
 * stalled segment between reliable updates) continues one precision up
 * from its iterate, as in eofa_solve; stats->inner_used reports it.
 * Arguments, outputs and errors as in eofa_solve. */
int eofa_solve_dense(eofa_ctx_t *ctx, double m1, double m2, const void *phi_dev, void *chiL_dev,
                     void *chiR_dev, void *Mphi_dev, double *S_out, const eofa_solver_t *solver,
                     eofa_stats_t *stats);

/* Rational approximation for the heatbath of Section 3.2: the best
 * relative-error approximation of x^(-1/2) on [lo, hi] of type (n, n),
 *   x^(-1/2) ~ alpha0 + sum_{l<n} alpha[l] / (beta[l] + x),
 * from Zolotarev's closed form (Jacobi elliptic functions by the
 * arithmetic-geometric mean).  The relative error alternates 2n + 2 times
 * on [lo, hi] with magnitude *delta_out (NULL: skip); every beta[l] > 0.
 * alpha/beta: caller-owned host arrays of n doubles.  Host computation
 * only, no context needed.  EOFA_EINVAL unless 0 < lo <= hi < inf and
 * 1 <= n <= 64. */
int eofa_rational_inv_sqrt(double lo, double hi, int n, double *alpha0, double *alpha,
                           double *beta, double *delta_out);

/* EOFA heatbath of eq. (3.1): phi ~ M_EOFA^(-1/2) eta, for a rational
 * approximation x^(-1/2) ~ alpha0 + sum_l alpha_l / (beta_l + x) and
 * gamma_l = 1 / (1 + beta_l):
 *   phi = alpha0 eta + sum_l alpha_l gamma_l { eta
 *       + k gamma_l P_- Omega_-^dag [H(m1) - gamma_l Delta_- P_-]^-1 Omega_- P_- eta
 *       - k gamma_l P_+ Omega_+^dag [H(m2) - gamma_l beta_l Delta_+ P_+]^-1 Omega_+ P_+ eta },
 * Delta_pm = k Omega_pm Omega_pm^dag (Omega, k as for eofa_solve).  Each
 * shifted operator is H(m+, m-) with one boundary mass moved: with
 * h(m) = m / N(m),
 *   H(m1) - g Delta_- P_- = H(m1, mL),  h(mL) = h(m1) + g (h(m2) - h(m1)),
 *   H(m2) - g Delta_+ P_+ = H(mR, m2),  h(mR) = h(m2) + g (h(m1) - h(m2)),
 * so the 2 n_poles inversions are Cayley-form even-odd solves as in
 * eofa_solve, to `solver`'s true-residual tolerance.
 *   eta_dev: 4D source (typically Gaussian), phi_dev: 4D output; device
 *   pointers, natural layout, may not alias.
 *   alpha/beta: caller-owned host arrays of n_poles doubles, beta_l > -1
 *   (n_poles = 0, or m1 = m2 where k = 0: phi = (alpha0 + sum_l alpha_l gamma_l) eta).
 *   forecast: chronological initial guesses (Section 5.2): each solve starts
 *   from the combination of the last `forecast` solutions of the same side
 *   that minimises its residual (Brower et al.); 0 starts every solve from
 *   zero.  0 <= forecast <= 16; the context then holds 3 * forecast extra
 *   FP64 half fields (2 GB each at 24^3x64, Ls = 24).
 *   stats (NULL: skip): iterations and reliable updates summed over the
 *   poles for the L (index 0) and R (index 1) side, true_resid the largest.
 * Requires m1 <= m2.  EOFA_ENOCONV if a solve missed the tolerance (phi is
 * still written); EOFA_EINVAL for bad arguments or a shift with N(m) <= 0. */
int eofa_heatbath(eofa_ctx_t *ctx, double m1, double m2, const void *eta_dev, int n_poles,
                  double alpha0, const double *alpha, const double *beta, int forecast,
                  void *phi_dev, const eofa_solver_t *solver, eofa_stats_t *stats);

/* Extreme eigenvalues of M_EOFA (eq. (2.5)), for choosing the interval of
 * the rational heatbath (Section 3.2): n_iter Lanczos steps from start_dev
 * (4D device field, natural layout; any nonzero vector), each applying
 * M_EOFA once, i.e. two Cayley-form solves with `solver` as in eofa_solve.
 *   theta_out[2]: the smallest and largest Ritz values;
 *   resid_out[2] (NULL: skip): their residual norms |M y - theta y| for the
 *   unit Ritz vectors y; an eigenvalue of M_EOFA lies within that distance
 *   of each Ritz value, and every Ritz value lies inside the spectrum (up
 *   to the solves' tolerance).
 *   stats (NULL: skip): solve iterations summed over the steps per side.
 * Requires m1 <= m2 and 2 <= n_iter <= 200.  Workspace: three 4D fields.
 * EOFA_ENOCONV if a solve missed the tolerance (outputs still written). */
int eofa_meofa_bounds(eofa_ctx_t *ctx, double m1, double m2, const void *start_dev, int n_iter,
                      const eofa_solver_t *solver, double *theta_out, double *resid_out,
                      eofa_stats_t *stats);

/* Chronological initial guesses across solves (the technique of Section 5.2,
 * Brower et al., applied to the molecular dynamics).  With depth > 0, every
 * solve of eofa_solve and eofa_force without an explicit initial guess
 * starts each EOFA system from the combination of that system's last
 * `depth` solutions (at the same masses) that minimises its residual with
 * the current links, and then adds its own solution to the history.
 * depth = 0 turns this off.  Every call clears the history: call it when the
 * pseudofermion changes (each trajectory).  0 <= depth <= 16; the context
 * then holds 3 * depth extra FP64 half fields.  With a history the
 * solutions depend on earlier calls, so molecular-dynamics reversibility
 * holds to the solver tolerance rather than to rounding. */
int eofa_chrono(eofa_ctx_t *ctx, int depth);

/* Pseudofermion force of eq. (3.2):
 *   d^a_{x,mu} S = k chi_L^dag g5 R5 (d^a D_w) chi_L - k chi_R^dag g5 R5 (d^a D_w) chi_R,
 * d^a the derivative along U_mu(x) -> exp(i eps T^a) U_mu(x), T^a = lambda^a/2.
 *   F_dev: F_mu(x) = sum_a T^a d^a S (Hermitian traceless 3x3 per link,
 *          gauge layout).  G_dev (NULL: skip): the complex-matrix gradient
 *          with dS = Re tr(G^dag dU) for any complex dU (gauge layout).
 *   chiL_dev/chiR_dev: solutions from eofa_solve; if either is NULL both
 *          are recomputed from phi_dev with `solver` (stats filled).
 * FP64 accumulation throughout. */
int eofa_force(eofa_ctx_t *ctx, double m1, double m2, const void *phi_dev,
               const void *chiL_dev, const void *chiR_dev, void *F_dev, void *G_dev,
               const eofa_solver_t *solver, eofa_stats_t *stats);

/* Molecular-dynamics update (HMC, Section 3), FP64, gauge layout:
 *   P <- P - dt_p F   (skipped if F_dev is NULL or dt_p == 0)
 *   U <- exp(i dt_u P) U  (skipped if dt_u == 0)
 * then kinetic_out (NULL: skip) = sum over links tr(P^2).
 * U_dev/P_dev are updated in place.  The context's own gauge copy is not
 * touched: call eofa_ctx_update_gauge afterwards. */
int eofa_md_update(eofa_ctx_t *ctx, void *U_dev, void *P_dev, const void *F_dev,
                   double dt_p, double dt_u, double *kinetic_out);

/* Allocation-free variant of eofa_md_update, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * molecular-dynamics loops, harnesses that forbid hipMalloc.  It performs
 * the same update with the same kernels and allocates nothing (no hipMalloc,
 * hipFree or allocating library call) and never synchronises:
 *   P <- P - dt_p F   (skipped if F_dev is NULL or dt_p == 0)
 *   U <- exp(i dt_u P) U  (skipped if dt_u == 0)
 *   *kinetic_dev = sum over links tr(P^2)   (NULL: skip)
 * kinetic_dev: one double in device memory (the caller's), written on the
 * context stream; it equals eofa_md_update's kinetic_out bit for bit.
 * The block partials of the kinetic sum live in a static device array of
 * 16384 doubles (128 KiB) that each GPU holds until the process ends, so a
 * kinetic sum needs V <= 1048576 4D sites (EOFA_EINVAL otherwise; without
 * kinetic_dev any size works).  All calls on one GPU share that array and
 * it keeps the last call's partials: calls with kinetic_dev that can
 * overlap on one GPU (different streams or threads without ordering) race.
 * Calls on one stream are ordered and safe.  No timing is recorded.
 * The context must have been created (eofa_ctx_create takes the array's
 * device address once per GPU).  Errors: EOFA_EINVAL (NULL ctx, U or P;
 * too large a lattice), EOFA_EDEVICE (launch failure). */
int eofa_md_update_noalloc(eofa_ctx_t *ctx, void *U_dev, void *P_dev, const void *F_dev,
                           double dt_p, double dt_u, double *kinetic_dev);

/* Gauge action of the ensembles the paper runs on (Table 1: Iwasaki), FP64:
 *   S_g = beta sum_x [ c0 sum_{mu<nu} (1 - Re tr W_1x1(x)/3)
 *                    + c1 sum_{mu!=nu} (1 - Re tr W_2x1(x)/3) ],  c0 = 1 - 8 c1,
 * W_1x1 the plaquette in the (mu, nu) plane at x and W_2x1 the loop two
 * links long in mu and one in nu.  c1 = -0.331: Iwasaki (the paper names the
 * action, not its coefficients); c1 = 0: Wilson.  Links are periodic in
 * every direction.
 * U_dev: any gauge field in the natural gauge layout (not necessarily the
 *        context's own copy); only the context's geometry and stream are used.
 * S_out: the action (host).  Synchronises the stream.
 * Errors: EOFA_EINVAL (NULL, non-finite beta or c1), EOFA_ENAN. */
int eofa_gauge_action(eofa_ctx_t *ctx, const void *U_dev, double beta, double c1, double *S_out);

/* Force of the gauge action above, in the convention of eofa_force:
 * F_mu(x) = sum_a T^a d^a S_g (Hermitian traceless 3x3 per link, gauge
 * layout), d^a along U_mu(x) -> exp(i eps T^a) U_mu(x), T^a = lambda^a/2.
 * accumulate = 0: F_dev = F_g; otherwise F_dev += F_g (to add the gauge
 * force to a fermion force).  F_dev must not alias U_dev.  Asynchronous
 * on the context stream.  Errors: EOFA_EINVAL (NULL, aliasing, non-finite). */
int eofa_gauge_force(eofa_ctx_t *ctx, const void *U_dev, double beta, double c1, void *F_dev, int accumulate);

/* Per-kernel timing with HIP events on the context stream.
 * eofa_timing_enable(ctx, 1) starts recording (and clears totals);
 * eofa_timing_query synchronises and returns, for kernel class `name`
 * ("hop" = the 5D hopping kernel in any precision, "hop64", "hop32",
 * "hop16", "hopb16", "blas", "force", "md", "gauge_force",
 * "gauge_action", "hop_dense" = the hopping kernel of eofa_solve_dense in
 * any of its precisions), the launch count, the summed duration in ms and
 * the summed algorithmic bytes. */
int eofa_timing_enable(eofa_ctx_t *ctx, int on);
int eofa_timing_query(eofa_ctx_t *ctx, const char *name, long *count, double *ms, double *bytes);

/* Message describing the last error on the calling thread ("" if none). */
const char *eofa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EOFA_H */
