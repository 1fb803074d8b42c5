/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the EOFA hot path of
 * D. Murphy, "Domain Wall Fermion Simulations with the Exact One-Flavor
 * Algorithm" (LATTICE 2016, arXiv:1611.00298).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source, header, table or helper with the GPU path.
 *
 * Every routine writes out a plain definition.  Where the paper is silent
 * (gamma basis, Wilson sign convention, boundary conditions, the closed
 * forms of k and Omega) the readings used are:
 *   - chiral gamma basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *     gamma_t = [[0,1],[1,0]], gamma_5 = gamma_x gamma_y gamma_z gamma_t;
 *   - D_w psi(x) = (4-M5) psi(x)
 *       - 1/2 sum_mu [(1-gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu)],
 *     antiperiodic in t (optional), periodic in space;
 *   - L = P+ L+(m+) + P- L-(m-), (L+ v)_s = v_{s-1}, (L+ v)_0 = -m+ v_{Ls-1},
 *     (L- v)_s = v_{s+1}, (L- v)_{Ls-1} = -m- v_0;
 *   - D_DWF = D_w (b5 + c5 L) + (1 - L)  (Section 2, eq. (2.3)), with the
 *     paper's c+d -> b5 and c-d -> c5.
 *
 * Layout (natural, lexicographic):
 *   4D site index  i = x + Lx*(y + Ly*(z + Lz*t))
 *   spinor site    12 complex numbers, [spin*3 + colour]
 *   5D field       [s][i][spin][colour]
 *   gauge field    [mu][i][a][b]
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int L[4];            /* Lx, Ly, Lz, Lt */
    int Ls;
    int antiperiodic_t;
    double M5;
    double b5, c5;       /* (c+d), (c-d) of eq. (2.3) */
} og_t;

/* ------------------------------------------------------------------ */
/* gamma matrices (chiral basis)                                        */
/* ------------------------------------------------------------------ */

static void gamma_matrix(int mu, cplx G[4][4])
{
    memset(G, 0, sizeof(cplx) * 16);
    if (mu == 3) {                       /* gamma_t = [[0,1],[1,0]] */
        G[0][2] = 1; G[1][3] = 1; G[2][0] = 1; G[3][1] = 1;
        return;
    }
    /* sigma_k */
    cplx s[2][2] = {{0, 0}, {0, 0}};
    if (mu == 0) { s[0][1] = 1; s[1][0] = 1; }
    if (mu == 1) { s[0][1] = -I; s[1][0] = I; }
    if (mu == 2) { s[0][0] = 1; s[1][1] = -1; }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            G[a][2 + b] = -I * s[a][b];  /* upper right: -i sigma_k */
            G[2 + a][b] = I * s[a][b];   /* lower left:  +i sigma_k */
        }
}

static void gamma5_matrix(cplx G5[4][4])
{
    cplx A[4][4], B[4][4], T[4][4];
    gamma_matrix(0, A);
    for (int mu = 1; mu < 4; mu++) {
        gamma_matrix(mu, B);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx acc = 0;
                for (int k = 0; k < 4; k++) acc += A[i][k] * B[k][j];
                T[i][j] = acc;
            }
        memcpy(A, T, sizeof(T));
    }
    memcpy(G5, A, sizeof(A));
}

/* exported for the convention tests: mu = 0..3 gamma_mu, mu = 4 gamma_5 */
void orc_gamma(int mu, double *out /* 16 complex, row major */)
{
    cplx G[4][4];
    if (mu == 4) gamma5_matrix(G); else gamma_matrix(mu, G);
    memcpy(out, G, sizeof(G));
}

/* out = (1 + sgn * gamma_mu) v on one spinor (12 complex) */
static void spin_proj(int mu, double sgn, const cplx *v, cplx *out)
{
    cplx G[4][4];
    gamma_matrix(mu, G);
    for (int a = 0; a < 4; a++)
        for (int c = 0; c < 3; c++) {
            cplx acc = v[a * 3 + c];
            for (int b = 0; b < 4; b++) acc += sgn * G[a][b] * v[b * 3 + c];
            out[a * 3 + c] = acc;
        }
}

/* out = M v for a 4x4 spin matrix M on one spinor */
static void spin_mat(cplx M[4][4], const cplx *v, cplx *out)
{
    for (int a = 0; a < 4; a++)
        for (int c = 0; c < 3; c++) {
            cplx acc = 0;
            for (int b = 0; b < 4; b++) acc += M[a][b] * v[b * 3 + c];
            out[a * 3 + c] = acc;
        }
}

/* chiral projector P_(+/-) = (1 +/- gamma_5)/2 as a spin matrix */
static void chiral_projector(int plus, cplx P[4][4])
{
    cplx G5[4][4];
    gamma5_matrix(G5);
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            P[a][b] = 0.5 * ((a == b ? 1.0 : 0.0) + (plus ? 1.0 : -1.0) * G5[a][b]);
}

/* ------------------------------------------------------------------ */
/* lattice geometry                                                     */
/* ------------------------------------------------------------------ */

static long vol4(const og_t *g) { return (long)g->L[0] * g->L[1] * g->L[2] * g->L[3]; }

static void coords(const og_t *g, long i, int c[4])
{
    for (int mu = 0; mu < 4; mu++) { c[mu] = (int)(i % g->L[mu]); i /= g->L[mu]; }
}

static long index4(const og_t *g, const int c[4])
{
    return c[0] + (long)g->L[0] * (c[1] + (long)g->L[1] * (c[2] + (long)g->L[2] * c[3]));
}

/* neighbour of site i in direction mu (dir = +1/-1); *sign picks up the
 * antiperiodic factor for hops across the time boundary */
static long neighbour(const og_t *g, long i, int mu, int dir, double *sign)
{
    int c[4];
    coords(g, i, c);
    *sign = 1.0;
    c[mu] += dir;
    if (c[mu] >= g->L[mu]) { c[mu] -= g->L[mu]; if (mu == 3 && g->antiperiodic_t) *sign = -1.0; }
    if (c[mu] < 0)         { c[mu] += g->L[mu]; if (mu == 3 && g->antiperiodic_t) *sign = -1.0; }
    return index4(g, c);
}

static int parity(const og_t *g, long i)
{
    int c[4];
    coords(g, i, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* ------------------------------------------------------------------ */
/* Wilson-Dirac operator D_w (Section 2, eq. (2.3))                      */
/* ------------------------------------------------------------------ */

/* colour multiply: out_spin = U v_spin (dag = 0) or U^dag v_spin (dag = 1) */
static void colour_mul(const cplx *U, int dag, const cplx *v, cplx *out)
{
    for (int sp = 0; sp < 4; sp++)
        for (int a = 0; a < 3; a++) {
            cplx acc = 0;
            for (int b = 0; b < 3; b++)
                acc += (dag ? conj(U[b * 3 + a]) : U[a * 3 + b]) * v[sp * 3 + b];
            out[sp * 3 + a] = acc;
        }
}

/* D_w (dagger = 0) or its adjoint (dagger = 1) at one site of one 4D slice.
 * The adjoint of the hopping terms exchanges (1-gamma) and (1+gamma). */
static void wilson_site(const og_t *g, const cplx *U, const cplx *in, long i,
                        int dagger, cplx *out)
{
    const long V = vol4(g);
    const double diag = 4.0 - g->M5;
    const double sf = dagger ? +1.0 : -1.0;   /* forward projector 1 + sf*gamma */
    const double sb = dagger ? -1.0 : +1.0;   /* backward projector 1 + sb*gamma */
    for (int k = 0; k < 12; k++) out[k] = diag * in[i * 12 + k];
    for (int mu = 0; mu < 4; mu++) {
        cplx v[12], w[12];
        double sgn;
        long jf = neighbour(g, i, mu, +1, &sgn);
        colour_mul(U + ((long)mu * V + i) * 9, 0, in + jf * 12, v);
        spin_proj(mu, sf, v, w);
        for (int k = 0; k < 12; k++) out[k] -= 0.5 * sgn * w[k];
        long jb = neighbour(g, i, mu, -1, &sgn);
        colour_mul(U + ((long)mu * V + jb) * 9, 1, in + jb * 12, v);
        spin_proj(mu, sb, v, w);
        for (int k = 0; k < 12; k++) out[k] -= 0.5 * sgn * w[k];
    }
}

/* D_w applied to nslice consecutive 4D slices (5D fields are s-diagonal) */
void orc_wilson(const og_t *g, const double *U_, const double *in_, double *out_,
                int nslice, int dagger)
{
    const cplx *U = (const cplx *)U_;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = vol4(g);
    for (int s = 0; s < nslice; s++) {
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < V; i++)
            wilson_site(g, U, in + (long)s * V * 12, i, dagger, out + ((long)s * V + i) * 12);
    }
}

/* ------------------------------------------------------------------ */
/* 5D hopping L (Section 2) and Ls x Ls matrices per chirality           */
/* ------------------------------------------------------------------ */

/* L (transpose = 0) or L^T (transpose = 1) on a 5D field.
 * L = P+ L+ + P- L-; L+ shifts s -> s-1 with -m+ on the wrap, L- shifts
 * s -> s+1 with -m- on the wrap.  L+^T and L-^T shift the other way. */
void orc_L(const og_t *g, double mp, double mm, int transpose,
           const double *in_, double *out_)
{
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = vol4(g);
    const int Ls = g->Ls;
    cplx Pp[4][4], Pm[4][4];
    chiral_projector(1, Pp);
    chiral_projector(0, Pm);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        for (int s = 0; s < Ls; s++) {
            /* shift towards lower s ("down"): source s-1, wrap factor -m */
            int sd = (s == 0) ? Ls - 1 : s - 1;
            /* shift towards higher s ("up"): source s+1, wrap factor -m */
            int su = (s == Ls - 1) ? 0 : s + 1;
            double fdp = (s == 0) ? -mp : 1.0, fdm = (s == 0) ? -mm : 1.0;
            double fup = (s == Ls - 1) ? -mp : 1.0, fum = (s == Ls - 1) ? -mm : 1.0;
            cplx vp[12], vm[12], a[12], b[12];
            const cplx *down = in + ((long)sd * V + i) * 12;
            const cplx *up = in + ((long)su * V + i) * 12;
            if (!transpose) {
                for (int k = 0; k < 12; k++) { vp[k] = fdp * down[k]; vm[k] = fum * up[k]; }
            } else {
                for (int k = 0; k < 12; k++) { vp[k] = fup * up[k]; vm[k] = fdm * down[k]; }
            }
            spin_mat(Pp, vp, a);
            spin_mat(Pm, vm, b);
            cplx *o = out + ((long)s * V + i) * 12;
            for (int k = 0; k < 12; k++) o[k] = a[k] + b[k];
        }
    }
}

/* The Ls x Ls matrix of L+ (plus = 1) or L- (plus = 0), row major */
static void L_matrix(int Ls, int plus, double m, double *A)
{
    memset(A, 0, sizeof(double) * Ls * Ls);
    for (int s = 0; s < Ls; s++) {
        if (plus) { if (s >= 1) A[s * Ls + s - 1] = 1.0; else A[0 * Ls + Ls - 1] = -m; }
        else      { if (s <= Ls - 2) A[s * Ls + s + 1] = 1.0; else A[(Ls - 1) * Ls + 0] = -m; }
    }
}

/* Gauss-Jordan inverse with partial pivoting of a real n x n matrix */
static int invert(int n, const double *A, double *Ainv)
{
    double *W = malloc(sizeof(double) * n * 2 * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++)
            W[i * 2 * n + j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(W[r * 2 * n + c]) > fabs(W[p * 2 * n + c])) p = r;
        if (W[p * 2 * n + c] == 0.0) { free(W); return -1; }
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                double t = W[c * 2 * n + j]; W[c * 2 * n + j] = W[p * 2 * n + j]; W[p * 2 * n + j] = t;
            }
        double d = W[c * 2 * n + c];
        for (int j = 0; j < 2 * n; j++) W[c * 2 * n + j] /= d;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double f = W[r * 2 * n + c];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; j++) W[r * 2 * n + j] -= f * W[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = W[i * 2 * n + n + j];
    free(W);
    return 0;
}

static void matmul(int n, const double *A, const double *B, double *C)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double acc = 0;
            for (int k = 0; k < n; k++) acc += A[i * n + k] * B[k * n + j];
            C[i * n + j] = acc;
        }
}

/* Named per-chirality Ls x Ls operators.  which:
 *   0: L            1: Dtilde = b5 + c5 L        2: Dtilde^-1
 *   3: D_perp = (1 - L) Dtilde^-1 (eq. (2.3))
 *   4: M_ee = (4 - M5) Dtilde + 1 - L  (the even-even block of D_DWF)
 *   5: M_ee^-1
 * A must hold Ls*Ls doubles; plus selects the P+ (m+) or P- (m-) block. */
int orc_chiral_matrix(const og_t *g, int which, int plus, double m, double *A)
{
    const int n = g->Ls;
    double *Lm = malloc(sizeof(double) * n * n), *Dt = malloc(sizeof(double) * n * n);
    double *T = malloc(sizeof(double) * n * n);
    int rc = 0;
    L_matrix(n, plus, m, Lm);
    for (int i = 0; i < n * n; i++) Dt[i] = g->c5 * Lm[i] + ((i / n == i % n) ? g->b5 : 0.0);
    switch (which) {
    case 0: memcpy(A, Lm, sizeof(double) * n * n); break;
    case 1: memcpy(A, Dt, sizeof(double) * n * n); break;
    case 2: rc = invert(n, Dt, A); break;
    case 3:
        rc = invert(n, Dt, T);
        for (int i = 0; i < n * n; i++) Lm[i] = ((i / n == i % n) ? 1.0 : 0.0) - Lm[i];
        matmul(n, Lm, T, A);
        break;
    case 4: case 5:
        for (int i = 0; i < n * n; i++)
            T[i] = (4.0 - g->M5) * Dt[i] + ((i / n == i % n) ? 1.0 : 0.0) - Lm[i];
        if (which == 4) memcpy(A, T, sizeof(double) * n * n);
        else rc = invert(n, T, A);
        break;
    default: rc = -1;
    }
    free(Lm); free(Dt); free(T);
    return rc;
}

/* out = P+ (A+ in) + P- (A- in) where A+/- act on s (transpose optional) */
static void apply_chiral(const og_t *g, const double *Ap, const double *Am, int transpose,
                         const cplx *in, cplx *out)
{
    const long V = vol4(g);
    const int Ls = g->Ls;
    cplx Pp[4][4], Pm[4][4];
    chiral_projector(1, Pp);
    chiral_projector(0, Pm);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        for (int s = 0; s < Ls; s++) {
            cplx vp[12] = {0}, vm[12] = {0}, a[12], b[12];
            for (int t = 0; t < Ls; t++) {
                double ap = transpose ? Ap[t * Ls + s] : Ap[s * Ls + t];
                double am = transpose ? Am[t * Ls + s] : Am[s * Ls + t];
                if (ap == 0.0 && am == 0.0) continue;
                const cplx *src = in + ((long)t * V + i) * 12;
                for (int k = 0; k < 12; k++) { vp[k] += ap * src[k]; vm[k] += am * src[k]; }
            }
            spin_mat(Pp, vp, a);
            spin_mat(Pm, vm, b);
            cplx *o = out + ((long)s * V + i) * 12;
            for (int k = 0; k < 12; k++) o[k] = a[k] + b[k];
        }
    }
}

/* Apply a named chiral operator (see orc_chiral_matrix) to a 5D field */
int orc_apply_chiral(const og_t *g, int which, double mp, double mm, int transpose,
                     const double *in, double *out)
{
    const int n = g->Ls;
    double *Ap = malloc(sizeof(double) * n * n), *Am = malloc(sizeof(double) * n * n);
    int rc = orc_chiral_matrix(g, which, 1, mp, Ap);
    rc |= orc_chiral_matrix(g, which, 0, mm, Am);
    if (!rc) apply_chiral(g, Ap, Am, transpose, (const cplx *)in, (cplx *)out);
    free(Ap); free(Am);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Moebius domain wall operator and the EOFA kernel (Section 2)          */
/* ------------------------------------------------------------------ */

static cplx *alloc5(const og_t *g) { return calloc((size_t)vol4(g) * g->Ls * 12, sizeof(cplx)); }
static long len5(const og_t *g) { return vol4(g) * g->Ls * 12; }

/* D_DWF(m+, m-) = D_w (b5 + c5 L) + (1 - L), eq. (2.3); dagger = adjoint,
 * (b5 + c5 L^T) D_w^dag + (1 - L^T). */
void orc_ddwf(const og_t *g, const double *U, double mp, double mm, int dagger,
              const double *in_, double *out_)
{
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long n = len5(g);
    cplx *Lin = alloc5(g), *tmp = alloc5(g);
    orc_L(g, mp, mm, dagger, in_, (double *)Lin);
    if (!dagger) {
        for (long k = 0; k < n; k++) tmp[k] = g->b5 * in[k] + g->c5 * Lin[k];
        orc_wilson(g, U, (const double *)tmp, out_, g->Ls, 0);
        for (long k = 0; k < n; k++) out[k] += in[k] - Lin[k];
    } else {
        cplx *Lt = alloc5(g);
        orc_wilson(g, U, in_, (double *)tmp, g->Ls, 1);
        orc_L(g, mp, mm, 1, (const double *)tmp, (double *)Lt);
        for (long k = 0; k < n; k++) out[k] = g->b5 * tmp[k] + g->c5 * Lt[k] + in[k] - Lin[k];
        free(Lt);
    }
    free(Lin); free(tmp);
}

/* D_EOFA = D_w + D_perp (eq. (2.3)); D_perp is dense in s */
void orc_deofa(const og_t *g, const double *U, double mp, double mm,
               const double *in_, double *out_)
{
    const long n = len5(g);
    cplx *t = alloc5(g);
    orc_wilson(g, U, in_, out_, g->Ls, 0);
    orc_apply_chiral(g, 3, mp, mm, 0, in_, (double *)t);
    cplx *out = (cplx *)out_;
    for (long k = 0; k < n; k++) out[k] += t[k];
    free(t);
}

/* gamma_5 R_5 on a 5D field: (R5 psi)_s = psi_{Ls-1-s} */
void orc_g5r5(const og_t *g, const double *in_, double *out_)
{
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = vol4(g);
    cplx G5[4][4];
    gamma5_matrix(G5);
    for (int s = 0; s < g->Ls; s++)
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < V; i++)
            spin_mat(G5, in + ((long)(g->Ls - 1 - s) * V + i) * 12, out + ((long)s * V + i) * 12);
}

/* H = gamma_5 R_5 D_EOFA(m+, m-) (Section 2) */
void orc_H(const og_t *g, const double *U, double mp, double mm,
           const double *in_, double *out_)
{
    cplx *t = alloc5(g);
    orc_deofa(g, U, mp, mm, in_, (double *)t);
    orc_g5r5(g, (const double *)t, out_);
    free(t);
}

/* ------------------------------------------------------------------ */
/* Omega, k  (Section 2: Delta_(+/-) = k Omega Omega^dag)                 */
/* ------------------------------------------------------------------ */

/* N(m) = b5^Ls + m (-c5)^Ls; Omega_-(s) = (-c5/b5)^s; Omega_+ = R5 Omega_-;
 * k = (b5 + c5) b5^(2Ls-2) (m2 - m1) / (N(m1) N(m2)).
 * These closed forms are a reading of the rank-one statement; the tests
 * compare k Omega Omega^T with R5 (D_perp(m2) - D_perp(m1)) built from
 * dense matrices. */
void orc_omega_k(const og_t *g, double m1, double m2, double *om_minus,
                 double *om_plus, double *k)
{
    const int Ls = g->Ls;
    const double b5 = g->b5, c5 = g->c5;
    double N1 = pow(b5, Ls) + m1 * pow(-c5, Ls);
    double N2 = pow(b5, Ls) + m2 * pow(-c5, Ls);
    for (int s = 0; s < Ls; s++) {
        om_minus[s] = pow(-c5 / b5, s);
        om_plus[Ls - 1 - s] = om_minus[s];
    }
    *k = (b5 + c5) * pow(b5, 2 * Ls - 2) * (m2 - m1) / (N1 * N2);
}

/* (Omega phi)(x,s) = Omega(s) P phi(x), P = P_- (minus = 1) or P_+ */
static void embed(const og_t *g, const double *om, int minus, const cplx *phi, cplx *out)
{
    const long V = vol4(g);
    cplx P[4][4];
    chiral_projector(!minus, P);
    for (long i = 0; i < V; i++) {
        cplx pp[12];
        spin_mat(P, phi + i * 12, pp);
        for (int s = 0; s < g->Ls; s++)
            for (int k = 0; k < 12; k++) out[((long)s * V + i) * 12 + k] = om[s] * pp[k];
    }
}

/* ------------------------------------------------------------------ */
/* linear algebra helpers                                               */
/* ------------------------------------------------------------------ */

static double norm2(long n, const cplx *a)
{
    double acc = 0;
    for (long k = 0; k < n; k++) acc += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return acc;
}

static cplx dot(long n, const cplx *a, const cplx *b)
{
    cplx acc = 0;
    for (long k = 0; k < n; k++) acc += conj(a[k]) * b[k];
    return acc;
}

typedef void (*op_fn)(void *ctx, const cplx *in, cplx *out);

/* CGNR (conjugate gradient on the normal equations A^dag A x = A^dag b,
 * with r = b - A x tracked explicitly).  Stops when |r|/|bnorm| < tol or
 * after fixed iterations when fixed > 0.  x is the initial guess. */
static int cgnr(op_fn A, op_fn Ad, void *ctx, long n, const cplx *b, cplx *x,
                double bnorm, double tol, int maxiter, int fixed, double *rres)
{
    cplx *r = calloc(n, sizeof(cplx)), *z = calloc(n, sizeof(cplx));
    cplx *p = calloc(n, sizeof(cplx)), *w = calloc(n, sizeof(cplx));
    A(ctx, x, w);
    for (long k = 0; k < n; k++) r[k] = b[k] - w[k];
    Ad(ctx, r, z);
    memcpy(p, z, n * sizeof(cplx));
    double zz = norm2(n, z), rr = norm2(n, r);
    int it = 0;
    for (;;) {
        if (fixed > 0) { if (it >= fixed) break; }
        else if (sqrt(rr) <= tol * bnorm || it >= maxiter) break;
        A(ctx, p, w);
        double ww = norm2(n, w);
        double alpha = zz / ww;
        for (long k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * w[k]; }
        rr = norm2(n, r);
        Ad(ctx, r, z);
        double zz_new = norm2(n, z);
        double beta = zz_new / zz;
        zz = zz_new;
        for (long k = 0; k < n; k++) p[k] = z[k] + beta * p[k];
        it++;
    }
    if (rres) *rres = sqrt(rr) / bnorm;
    free(r); free(z); free(p); free(w);
    return it;
}

/* ------------------------------------------------------------------ */
/* even-odd (red-black) Schur complement (Section 5.1)                  */
/* ------------------------------------------------------------------ */

static void mask_parity(const og_t *g, int par, const cplx *in, cplx *out)
{
    const long V = vol4(g);
    for (int s = 0; s < g->Ls; s++)
        for (long i = 0; i < V; i++) {
            int keep = parity(g, i) == par;
            for (int k = 0; k < 12; k++)
                out[((long)s * V + i) * 12 + k] = keep ? in[((long)s * V + i) * 12 + k] : 0;
        }
}

typedef struct { const og_t *g; const double *U; double mp, mm; } opctx_t;

/* Mhat = M_oo - M_oe M_ee^-1 M_eo on odd sites, blocks taken from D_DWF by
 * parity masks; Mhat^dag uses the blocks of D_DWF^dag.  in/out are full
 * 5D fields; even sites of in are ignored, even sites of out are zero. */
void orc_schur(const og_t *g, const double *U, double mp, double mm, int dagger,
               const double *in_, double *out_)
{
    cplx *x = alloc5(g), *t = alloc5(g), *a = alloc5(g), *u = alloc5(g);
    mask_parity(g, 1, (const cplx *)in_, x);
    orc_ddwf(g, U, mp, mm, dagger, (const double *)x, (double *)t);   /* t_o = M_oo x, t_e = M_eo x */
    mask_parity(g, 0, t, a);
    orc_apply_chiral(g, 5, mp, mm, dagger, (const double *)a, (double *)u);  /* M_ee^-1 (or ^-dag) */
    orc_ddwf(g, U, mp, mm, dagger, (const double *)u, (double *)a);   /* a_o = M_oe u */
    const long n = len5(g);
    for (long k = 0; k < n; k++) t[k] -= a[k];
    mask_parity(g, 1, t, (cplx *)out_);
    free(x); free(t); free(a); free(u);
}

static void schur_op(void *c, const cplx *in, cplx *out)
{
    opctx_t *o = c;
    orc_schur(o->g, o->U, o->mp, o->mm, 0, (const double *)in, (double *)out);
}
static void schur_op_dag(void *c, const cplx *in, cplx *out)
{
    opctx_t *o = c;
    orc_schur(o->g, o->U, o->mp, o->mm, 1, (const double *)in, (double *)out);
}

/* Solve D_DWF(m+, m-) y = b by even-odd preconditioning and CGNR on the
 * odd-site Schur complement (Section 5.1):
 *   bhat_o = b_o - M_oe M_ee^-1 b_e,  Mhat y_o = bhat_o,
 *   y_e = M_ee^-1 (b_e - M_eo y_o).
 * Stops when |bhat - Mhat y_o| < tol |b| (or after `fixed` iterations).
 * Returns the iteration count; *resid = |b - D_DWF y| / |b|. */
int orc_solve_ddwf_eo(const og_t *g, const double *U, double mp, double mm,
                      const double *b_, double *y_, double tol, int maxiter,
                      int fixed, double *resid)
{
    const long n = len5(g);
    const cplx *b = (const cplx *)b_;
    cplx *y = (cplx *)y_;
    cplx *be = alloc5(g), *t = alloc5(g), *u = alloc5(g), *bh = alloc5(g), *x = alloc5(g);
    mask_parity(g, 0, b, be);
    orc_apply_chiral(g, 5, mp, mm, 0, (const double *)be, (double *)t);
    orc_ddwf(g, U, mp, mm, 0, (const double *)t, (double *)u);
    for (long k = 0; k < n; k++) t[k] = b[k] - u[k];
    mask_parity(g, 1, t, bh);
    opctx_t ctx = {g, U, mp, mm};
    double bnorm = sqrt(norm2(n, b));
    int it = cgnr(schur_op, schur_op_dag, &ctx, n, bh, x, bnorm, tol, maxiter, fixed, NULL);
    /* reconstruct the even sites */
    orc_ddwf(g, U, mp, mm, 0, (const double *)x, (double *)u);   /* u_e = M_eo y_o */
    for (long k = 0; k < n; k++) t[k] = b[k] - u[k];
    mask_parity(g, 0, t, be);
    orc_apply_chiral(g, 5, mp, mm, 0, (const double *)be, (double *)u);
    mask_parity(g, 0, u, t);
    for (long k = 0; k < n; k++) y[k] = x[k] + t[k];
    if (resid) {
        orc_ddwf(g, U, mp, mm, 0, (const double *)y, (double *)u);
        for (long k = 0; k < n; k++) u[k] = b[k] - u[k];
        *resid = sqrt(norm2(n, u)) / bnorm;
    }
    free(be); free(t); free(u); free(bh); free(x);
    return it;
}

static void H_op(void *c, const cplx *in, cplx *out)
{
    opctx_t *o = c;
    orc_H(o->g, o->U, o->mp, o->mm, (const double *)in, (double *)out);
}

/* Solve H(m+, m-) chi = v directly (H Hermitian, dense D_perp in s) by
 * CGNR; stops when |v - H chi| < tol |v|.  This is the definition-level
 * path, with no Cayley form and no even-odd preconditioning. */
int orc_solve_H(const og_t *g, const double *U, double mp, double mm,
                const double *v_, double *chi_, double tol, int maxiter, double *resid)
{
    const long n = len5(g);
    opctx_t ctx = {g, U, mp, mm};
    memset(chi_, 0, n * sizeof(cplx));
    double vnorm = sqrt(norm2(n, (const cplx *)v_));
    return cgnr(H_op, H_op, &ctx, n, (const cplx *)v_, (cplx *)chi_, vnorm, tol, maxiter, 0, resid);
}

/* ------------------------------------------------------------------ */
/* heatbath operators of eq. (3.1)                                       */
/* ------------------------------------------------------------------ */

typedef struct { const og_t *g; const double *U; double m; double gk; const double *om; int minus; } shctx_t;

/* out = [H(m) - gk Omega Omega^dag P] in, with Omega Omega^dag P acting as
 * (Omega Omega^dag P psi)(x,s) = Omega(s) P sum_s' Omega(s') psi(x,s');
 * minus = 1: P_-, else P_+.  gk = g k for Delta = k Omega Omega^dag. */
static void shifted_op(void *c, const cplx *in, cplx *out)
{
    const shctx_t *o = c;
    const og_t *g = o->g;
    const long V = vol4(g);
    orc_H(g, o->U, o->m, o->m, (const double *)in, (double *)out);
    cplx P[4][4];
    chiral_projector(!o->minus, P);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx acc[12] = {0}, pa[12];
        for (int s = 0; s < g->Ls; s++)
            for (int k = 0; k < 12; k++) acc[k] += o->om[s] * in[((long)s * V + i) * 12 + k];
        spin_mat(P, acc, pa);
        for (int s = 0; s < g->Ls; s++)
            for (int k = 0; k < 12; k++) out[((long)s * V + i) * 12 + k] -= o->gk * o->om[s] * pa[k];
    }
}

/* which = 0: H(m1) - g Delta_- P_-;  which = 1: H(m2) - g Delta_+ P_+. */
void orc_H_shifted(const og_t *g, const double *U, double m1, double m2, int which, double gshift,
                   const double *in_, double *out_)
{
    double *om_m = malloc(sizeof(double) * g->Ls), *om_p = malloc(sizeof(double) * g->Ls), k;
    orc_omega_k(g, m1, m2, om_m, om_p, &k);
    shctx_t ctx = {g, U, which ? m2 : m1, gshift * k, which ? om_p : om_m, !which};
    shifted_op(&ctx, (const cplx *)in_, (cplx *)out_);
    free(om_m); free(om_p);
}

/* Solve the shifted system of orc_H_shifted for chi (CGNR; the operator is
 * Hermitian, so A^dag = A); stops when |v - A chi| < tol |v|. */
int orc_solve_H_shifted(const og_t *g, const double *U, double m1, double m2, int which,
                        double gshift, const double *v_, double *chi_, double tol, int maxiter,
                        double *resid)
{
    const long n = len5(g);
    double *om_m = malloc(sizeof(double) * g->Ls), *om_p = malloc(sizeof(double) * g->Ls), k;
    orc_omega_k(g, m1, m2, om_m, om_p, &k);
    shctx_t ctx = {g, U, which ? m2 : m1, gshift * k, which ? om_p : om_m, !which};
    memset(chi_, 0, n * sizeof(cplx));
    double vnorm = sqrt(norm2(n, (const cplx *)v_));
    int it = vnorm > 0 ? cgnr(shifted_op, shifted_op, &ctx, n, (const cplx *)v_, (cplx *)chi_, vnorm,
                              tol, maxiter, 0, resid) : 0;
    if (vnorm == 0 && resid) *resid = 0;
    free(om_m); free(om_p);
    return it;
}

/* ------------------------------------------------------------------ */
/* EOFA solutions, action and force (Sections 2, 3.1, 3.3 (force: eq. (3.2)))               */
/* ------------------------------------------------------------------ */

/* chi_L = H(m1,m1)^-1 Omega_- P_- phi and chi_R = H(m1,m2)^-1 Omega_+ P_+ phi
 * (eq. (3.2) definitions; H(m2) - Delta_+ P_+ = H(m+ = m1, m- = m2)).
 * method 0: direct solve with H.  method 1: Cayley form of the Section 5.1
 * footnote, chi = Dtilde D_DWF^-1 gamma_5 R_5 v, with the even-odd solve. */
int orc_eofa_chi(const og_t *g, const double *U, double m1, double m2,
                 const double *phi, double *chiL, double *chiR, int method,
                 double tol, int maxiter, int *iters)
{
    const int Ls = g->Ls;
    double *om_m = malloc(sizeof(double) * Ls), *om_p = malloc(sizeof(double) * Ls), k;
    orc_omega_k(g, m1, m2, om_m, om_p, &k);
    cplx *v = alloc5(g), *b = alloc5(g), *y = alloc5(g);
    int rc = 0;
    for (int sys = 0; sys < 2; sys++) {
        double mp = m1, mm = sys == 0 ? m1 : m2;
        double *chi = sys == 0 ? chiL : chiR;
        embed(g, sys == 0 ? om_m : om_p, sys == 0, (const cplx *)phi, v);
        int it;
        if (method == 0) {
            it = orc_solve_H(g, U, mp, mm, (const double *)v, chi, tol, maxiter, NULL);
        } else {
            orc_g5r5(g, (const double *)v, (double *)b);
            it = orc_solve_ddwf_eo(g, U, mp, mm, (const double *)b, (double *)y, tol, maxiter, 0, NULL);
            orc_apply_chiral(g, 1, mp, mm, 0, (const double *)y, chi);
        }
        if (iters) iters[sys] = it;
        if (it >= maxiter) rc = 1;
    }
    free(om_m); free(om_p); free(v); free(b); free(y);
    return rc;
}

/* S = phi^dag M_EOFA phi with M_EOFA of eq. (2.5):
 *   M_EOFA phi = phi - k P_- Omega_-^dag chi_L + k P_+ Omega_+^dag chi_R.
 * S[0] = Re S, S[1] = Im S (zero up to rounding).  Mphi may be NULL. */
void orc_action(const og_t *g, double m1, double m2, const double *phi_,
                const double *chiL_, const double *chiR_, double *S, double *Mphi_)
{
    const long V = vol4(g);
    const int Ls = g->Ls;
    const cplx *phi = (const cplx *)phi_, *chiL = (const cplx *)chiL_, *chiR = (const cplx *)chiR_;
    double *om_m = malloc(sizeof(double) * Ls), *om_p = malloc(sizeof(double) * Ls), k;
    orc_omega_k(g, m1, m2, om_m, om_p, &k);
    cplx Pp[4][4], Pm[4][4];
    chiral_projector(1, Pp);
    chiral_projector(0, Pm);
    cplx *M = calloc(V * 12, sizeof(cplx));
    for (long i = 0; i < V; i++) {
        cplx aL[12] = {0}, aR[12] = {0}, pL[12], pR[12];
        for (int s = 0; s < Ls; s++)
            for (int c = 0; c < 12; c++) {
                aL[c] += om_m[s] * chiL[((long)s * V + i) * 12 + c];
                aR[c] += om_p[s] * chiR[((long)s * V + i) * 12 + c];
            }
        spin_mat(Pm, aL, pL);
        spin_mat(Pp, aR, pR);
        for (int c = 0; c < 12; c++) M[i * 12 + c] = phi[i * 12 + c] - k * pL[c] + k * pR[c];
    }
    cplx s = dot(V * 12, phi, M);
    S[0] = creal(s);
    S[1] = cimag(s);
    if (Mphi_) memcpy(Mphi_, M, V * 12 * sizeof(cplx));
    free(M); free(om_m); free(om_p);
}

/* eta^dag (dD_w[dU]) chi for a variation dU of the single link U_mu(x):
 * D_w contains -1/2 (1-gamma_mu) U_mu(x) at (x, x+mu) and
 * -1/2 (1+gamma_mu) U_mu(x)^dag at (x+mu, x), times the boundary sign.
 * Summed over s, spin and colour; eta = gamma_5 R_5 chi. */
static cplx link_variation(const og_t *g, long i, int mu, const cplx *dU,
                           const cplx *chi, const cplx *eta)
{
    const long V = vol4(g);
    double sgn;
    long j = neighbour(g, i, mu, +1, &sgn);
    cplx acc = 0;
    for (int s = 0; s < g->Ls; s++) {
        cplx v[12], w[12];
        /* at x: -1/2 sgn (1-gamma) dU chi(x+mu) */
        colour_mul(dU, 0, chi + ((long)s * V + j) * 12, v);
        spin_proj(mu, -1.0, v, w);
        for (int c = 0; c < 12; c++) acc += conj(eta[((long)s * V + i) * 12 + c]) * (-0.5 * sgn * w[c]);
        /* at x+mu: -1/2 sgn (1+gamma) dU^dag chi(x) */
        colour_mul(dU, 1, chi + ((long)s * V + i) * 12, v);
        spin_proj(mu, +1.0, v, w);
        for (int c = 0; c < 12; c++) acc += conj(eta[((long)s * V + j) * 12 + c]) * (-0.5 * sgn * w[c]);
    }
    return acc;
}

/* Pseudofermion force of eq. (3.2):
 *   d^a_{x,mu} S = k chi_L^dag g5 R5 (d^a D_w) chi_L - k chi_R^dag g5 R5 (d^a D_w) chi_R
 * with d^a the derivative along U_mu(x) -> exp(i eps T^a) U_mu(x),
 * T^a = lambda^a / 2.  F_mu(x) = sum_a T^a d^a S (Hermitian, traceless).
 * G (may be NULL) is the complex-matrix gradient with
 *   dS = Re tr(G^dag dU) for any complex dU, built entry by entry.
 * links: NULL for every link, else nlinks pairs (mu, i); F and G are then
 * packed as [nlinks][3][3]. */
void orc_force(const og_t *g, const double *U_, double m1, double m2,
               const double *chiL_, const double *chiR_, double *F_, double *G_,
               const int *links, long nlinks)
{
    const long V = vol4(g);
    const int Ls = g->Ls;
    const cplx *U = (const cplx *)U_;
    double *om_m = malloc(sizeof(double) * Ls), *om_p = malloc(sizeof(double) * Ls), k;
    orc_omega_k(g, m1, m2, om_m, om_p, &k);
    free(om_m); free(om_p);
    cplx *etaL = alloc5(g), *etaR = alloc5(g);
    orc_g5r5(g, chiL_, (double *)etaL);
    orc_g5r5(g, chiR_, (double *)etaR);
    const cplx *chiL = (const cplx *)chiL_, *chiR = (const cplx *)chiR_;
    /* generators T^a = lambda^a / 2 */
    cplx T[8][9];
    memset(T, 0, sizeof(T));
    T[0][1] = T[0][3] = 0.5;
    T[1][1] = -0.5 * I; T[1][3] = 0.5 * I;
    T[2][0] = 0.5; T[2][4] = -0.5;
    T[3][2] = T[3][6] = 0.5;
    T[4][2] = -0.5 * I; T[4][6] = 0.5 * I;
    T[5][5] = T[5][7] = 0.5;
    T[6][5] = -0.5 * I; T[6][7] = 0.5 * I;
    T[7][0] = T[7][4] = 0.5 / sqrt(3.0); T[7][8] = -1.0 / sqrt(3.0);
    long nl = links ? nlinks : 4 * V;
    cplx *F = (cplx *)F_, *G = (cplx *)G_;
    #pragma omp parallel for schedule(dynamic, 16)
    for (long l = 0; l < nl; l++) {
        int mu = links ? links[2 * l] : (int)(l / V);
        long i = links ? links[2 * l + 1] : l % V;
        const cplx *Ul = U + ((long)mu * V + i) * 9;
        cplx Fl[9] = {0};
        for (int a = 0; a < 8; a++) {
            cplx dU[9];
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) {
                    cplx acc = 0;
                    for (int q = 0; q < 3; q++) acc += I * T[a][r * 3 + q] * Ul[q * 3 + c];
                    dU[r * 3 + c] = acc;
                }
            cplx d = k * link_variation(g, i, mu, dU, chiL, etaL)
                   - k * link_variation(g, i, mu, dU, chiR, etaR);
            double da = creal(d);
            for (int e = 0; e < 9; e++) Fl[e] += T[a][e] * da;
        }
        memcpy(F + l * 9, Fl, sizeof(Fl));
        if (G) {
            for (int e = 0; e < 9; e++) {
                cplx dU[9] = {0};
                dU[e] = 1.0;
                cplx dre = k * link_variation(g, i, mu, dU, chiL, etaL)
                         - k * link_variation(g, i, mu, dU, chiR, etaR);
                dU[e] = I;
                cplx dim = k * link_variation(g, i, mu, dU, chiL, etaL)
                         - k * link_variation(g, i, mu, dU, chiR, etaR);
                G[l * 9 + e] = creal(dre) + I * creal(dim);
            }
        }
    }
    free(etaL); free(etaR);
}

/* ------------------------------------------------------------------ */
/* single-site evaluation, for sampled checks on large lattices          */
/* ------------------------------------------------------------------ */

/* A field is read through a fetch callback returning the 12 complex
 * numbers at (i, s) (possibly computed into buf). */
typedef const cplx *(*fetch_fn)(void *ctx, long i, int s, cplx *buf);

typedef struct { const og_t *g; const cplx *f; int parity; } arr_ctx;

/* plain array; parity >= 0 masks the other parity to zero */
static const cplx *fetch_array(void *c, long i, int s, cplx *buf)
{
    arr_ctx *a = c;
    if (a->parity >= 0 && parity(a->g, i) != a->parity) {
        for (int k = 0; k < 12; k++) buf[k] = 0;
        return buf;
    }
    return a->f + ((long)s * vol4(a->g) + i) * 12;
}

static void wilson_at(const og_t *g, const cplx *U, fetch_fn f, void *c, long i, int s,
                      int dagger, cplx *out)
{
    const long V = vol4(g);
    const double diag = 4.0 - g->M5;
    const double sf = dagger ? +1.0 : -1.0, sb = dagger ? -1.0 : +1.0;
    cplx buf[12], v[12], w[12];
    const cplx *p = f(c, i, s, buf);
    for (int k = 0; k < 12; k++) out[k] = diag * p[k];
    for (int mu = 0; mu < 4; mu++) {
        double sgn;
        long jf = neighbour(g, i, mu, +1, &sgn);
        p = f(c, jf, s, buf);
        colour_mul(U + ((long)mu * V + i) * 9, 0, p, v);
        spin_proj(mu, sf, v, w);
        for (int k = 0; k < 12; k++) out[k] -= 0.5 * sgn * w[k];
        long jb = neighbour(g, i, mu, -1, &sgn);
        p = f(c, jb, s, buf);
        colour_mul(U + ((long)mu * V + jb) * 9, 1, p, v);
        spin_proj(mu, sb, v, w);
        for (int k = 0; k < 12; k++) out[k] -= 0.5 * sgn * w[k];
    }
}

static void L_at(const og_t *g, double mp, double mm, int transpose, fetch_fn f, void *c,
                 long i, int s, cplx *out)
{
    const int Ls = g->Ls;
    cplx Pp[4][4], Pm[4][4], vp[12], vm[12], a[12], b[12], b1[12], b2[12];
    chiral_projector(1, Pp);
    chiral_projector(0, Pm);
    int sd = (s == 0) ? Ls - 1 : s - 1, su = (s == Ls - 1) ? 0 : s + 1;
    double fdp = (s == 0) ? -mp : 1.0, fdm = (s == 0) ? -mm : 1.0;
    double fup = (s == Ls - 1) ? -mp : 1.0, fum = (s == Ls - 1) ? -mm : 1.0;
    const cplx *down = f(c, i, sd, b1), *up = f(c, i, su, b2);
    for (int k = 0; k < 12; k++) {
        if (!transpose) { vp[k] = fdp * down[k]; vm[k] = fum * up[k]; }
        else            { vp[k] = fup * up[k];   vm[k] = fdm * down[k]; }
    }
    spin_mat(Pp, vp, a);
    spin_mat(Pm, vm, b);
    for (int k = 0; k < 12; k++) out[k] = a[k] + b[k];
}

typedef struct { const og_t *g; const cplx *U; double mp, mm; fetch_fn f; void *c; } dctx;

/* (b5 + c5 L) psi at one site */
static const cplx *fetch_dtilde(void *cv, long i, int s, cplx *buf)
{
    dctx *d = cv;
    cplx b1[12], Lv[12];
    const cplx *p = d->f(d->c, i, s, b1);
    L_at(d->g, d->mp, d->mm, 0, d->f, d->c, i, s, Lv);
    for (int k = 0; k < 12; k++) buf[k] = d->g->b5 * p[k] + d->g->c5 * Lv[k];
    return buf;
}

/* D_w^dag psi at one site */
static const cplx *fetch_wdag(void *cv, long i, int s, cplx *buf)
{
    dctx *d = cv;
    wilson_at(d->g, d->U, d->f, d->c, i, s, 1, buf);
    return buf;
}

/* (D_DWF psi)(i, s) or (D_DWF^dag psi)(i, s), same formulas as orc_ddwf */
static void ddwf_at(const og_t *g, const cplx *U, double mp, double mm, int dagger,
                    fetch_fn f, void *c, long i, int s, cplx *out)
{
    dctx d = {g, U, mp, mm, f, c};
    cplx b1[12], Lv[12];
    const cplx *p = f(c, i, s, b1);
    if (!dagger) {
        wilson_at(g, U, fetch_dtilde, &d, i, s, 0, out);
        L_at(g, mp, mm, 0, f, c, i, s, Lv);
        for (int k = 0; k < 12; k++) out[k] += p[k] - Lv[k];
    } else {
        cplx w[12], Lw[12];
        fetch_wdag(&d, i, s, w);
        L_at(g, mp, mm, 1, fetch_wdag, &d, i, s, Lw);
        L_at(g, mp, mm, 1, f, c, i, s, Lv);
        for (int k = 0; k < 12; k++) out[k] = g->b5 * w[k] + g->c5 * Lw[k] + p[k] - Lv[k];
    }
}

/* (D_DWF psi)(i, s) at a list of (s, i) pairs; out is [n][12] complex */
void orc_ddwf_sites(const og_t *g, const double *U_, double mp, double mm, int dagger,
                    const double *in_, const long *sites, long n, double *out_)
{
    arr_ctx a = {g, (const cplx *)in_, -1};
    #pragma omp parallel for schedule(dynamic, 4)
    for (long q = 0; q < n; q++)
        ddwf_at(g, (const cplx *)U_, mp, mm, dagger, fetch_array, &a,
                sites[2 * q + 1], (int)sites[2 * q], (cplx *)out_ + q * 12);
}

/* cached values of a = M_ee^-1 (or ^-dag) [D psi_o]_e on the 9 sites around
 * one odd site, all s */
typedef struct { const og_t *g; long site[9]; cplx *val; } cache_ctx;

static const cplx *fetch_cache(void *cv, long i, int s, cplx *buf)
{
    cache_ctx *c = cv;
    for (int j = 0; j < 9; j++)
        if (c->site[j] == i) return c->val + ((long)j * c->g->Ls + s) * 12;
    for (int k = 0; k < 12; k++) buf[k] = 0;   /* not reached for the stencil */
    return buf;
}

/* (Mhat psi)(i, s) or (Mhat^dag psi)(i, s) at odd sites i, as orc_schur */
void orc_schur_sites(const og_t *g, const double *U_, double mp, double mm, int dagger,
                     const double *in_, const long *sites, long n, double *out_)
{
    const int Ls = g->Ls;
    const cplx *U = (const cplx *)U_;
    double *Ap = malloc(sizeof(double) * Ls * Ls), *Am = malloc(sizeof(double) * Ls * Ls);
    orc_chiral_matrix(g, 5, 1, mp, Ap);
    orc_chiral_matrix(g, 5, 0, mm, Am);
    cplx Pp[4][4], Pm[4][4];
    chiral_projector(1, Pp);
    chiral_projector(0, Pm);
    arr_ctx odd = {g, (const cplx *)in_, 1};
    #pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < n; q++) {
        int s = (int)sites[2 * q];
        long i = sites[2 * q + 1];
        cache_ctx cc;
        cc.g = g;
        cc.val = calloc((size_t)9 * Ls * 12, sizeof(cplx));
        cplx *t = calloc((size_t)Ls * 12, sizeof(cplx));
        cc.site[0] = i;
        for (int mu = 0; mu < 4; mu++) {
            double sg;
            cc.site[1 + 2 * mu] = neighbour(g, i, mu, +1, &sg);
            cc.site[2 + 2 * mu] = neighbour(g, i, mu, -1, &sg);
        }
        for (int j = 1; j < 9; j++) {
            long y = cc.site[j];
            for (int s2 = 0; s2 < Ls; s2++)
                ddwf_at(g, U, mp, mm, dagger, fetch_array, &odd, y, s2, t + (long)s2 * 12);
            for (int s1 = 0; s1 < Ls; s1++) {
                cplx vp[12] = {0}, vm[12] = {0}, a[12], b[12];
                for (int s2 = 0; s2 < Ls; s2++) {
                    double ap = dagger ? Ap[s2 * Ls + s1] : Ap[s1 * Ls + s2];
                    double am = dagger ? Am[s2 * Ls + s1] : Am[s1 * Ls + s2];
                    for (int k = 0; k < 12; k++) { vp[k] += ap * t[s2 * 12 + k]; vm[k] += am * t[s2 * 12 + k]; }
                }
                spin_mat(Pp, vp, a);
                spin_mat(Pm, vm, b);
                for (int k = 0; k < 12; k++) cc.val[((long)j * Ls + s1) * 12 + k] = a[k] + b[k];
            }
        }
        /* site 0 (odd) of the cache stays zero: a lives on even sites */
        cplx tt[12], uu[12];
        ddwf_at(g, U, mp, mm, dagger, fetch_array, &odd, i, s, tt);
        ddwf_at(g, U, mp, mm, dagger, fetch_cache, &cc, i, s, uu);
        for (int k = 0; k < 12; k++) ((cplx *)out_)[q * 12 + k] = tt[k] - uu[k];
        free(cc.val);
        free(t);
    }
    free(Ap); free(Am);
}
