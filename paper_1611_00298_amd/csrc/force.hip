// force.hip -- EOFA pseudofermion force (eq. (3.2)) and the MD link update.
//
// For a link U_mu(x) the variation of S = phi^dag M_EOFA phi is
//   k chi_L^dag g5 R5 (dD_w) chi_L - k chi_R^dag g5 R5 (dD_w) chi_R.
// With eta = g5 R5 chi and B[chi] = sum_{s,spin} chi_s(x) (x) ((1+gamma_mu) eta_s(x+mu))^dag
// the complex gradient (dS = Re tr(G^dag dU)) is G = -sigma k (B[chi_L] - B[chi_R]),
// and the su(3) force F = sum_a T^a d^a S is (1/4) TA(-i W) with
// W = sigma k (U B^dag - B U^dag), B = B[chi_L] - B[chi_R], sigma the
// boundary sign of the link.  Because (1+gamma_mu) has rank two,
// B = sum_{s} sum_{j=0,1} h_j (x) g_j^dag with h = chi_up + A_mu chi_lo at x
// and g = chi_up - A_mu chi_lo at (x+mu, Ls-1-s) (the minus sign is gamma_5).
// FP64 throughout; one work-item per link, fields in the natural layout.
#include "internal.h"

namespace eofa {

struct cplx {
    double r, i;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) { return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i}; }  // a conj(b)

// (A_mu v_lo)_j for the chiral-basis block A_mu of gamma_mu (see dslash.hip)
__device__ __forceinline__ void amul(int mu, cplx v2, cplx v3, cplx& o0, cplx& o1) {
    switch (mu) {
    case 0: o0 = {v3.i, -v3.r}; o1 = {v2.i, -v2.r}; break;     // -i v3, -i v2
    case 1: o0 = {-v3.r, -v3.i}; o1 = {v2.r, v2.i}; break;     // -v3, v2
    case 2: o0 = {v2.i, -v2.r}; o1 = {-v3.i, v3.r}; break;     // -i v2, i v3
    default: o0 = v2; o1 = v3; break;                          // v2, v3
    }
}

__global__ void __launch_bounds__(256) k_force(const double2* __restrict__ U,
                                               const double2* __restrict__ chiL,
                                               const double2* __restrict__ chiR, double k,
                                               double2* __restrict__ F, double2* __restrict__ G,
                                               int Lx, int Ly, int Lz, int Lt, int Ls, int aperiodic) {
    const int V = Lx * Ly * Lz * Lt;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= 4 * V) return;
    const int mu = l / V, i = l - mu * V;
    int c[4] = {i % Lx, (i / Lx) % Ly, (i / (Lx * Ly)) % Lz, i / (Lx * Ly * Lz)};
    const int L[4] = {Lx, Ly, Lz, Lt};
    double sigma = 1.0;
    c[mu] += 1;
    if (c[mu] == L[mu]) { c[mu] = 0; if (mu == 3 && aperiodic) sigma = -1.0; }
    const int j = c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]));

    cplx B[9];
    for (int q = 0; q < 9; ++q) B[q] = {0.0, 0.0};
    for (int sys = 0; sys < 2; ++sys) {
        const double2* chi = sys ? chiR : chiL;
        const double sg = sys ? -1.0 : 1.0;
        for (int s = 0; s < Ls; ++s) {
            const double2* a = chi + ((size_t)s * V + i) * 12;
            const double2* b = chi + ((size_t)(Ls - 1 - s) * V + j) * 12;
            cplx h[2][3], g[2][3];
            for (int cc = 0; cc < 3; ++cc) {
                cplx a0 = {a[cc].x, a[cc].y}, a1 = {a[3 + cc].x, a[3 + cc].y};
                cplx a2 = {a[6 + cc].x, a[6 + cc].y}, a3 = {a[9 + cc].x, a[9 + cc].y};
                cplx b0 = {b[cc].x, b[cc].y}, b1 = {b[3 + cc].x, b[3 + cc].y};
                cplx b2 = {b[6 + cc].x, b[6 + cc].y}, b3 = {b[9 + cc].x, b[9 + cc].y};
                cplx p0, p1, q0, q1;
                amul(mu, a2, a3, p0, p1);
                amul(mu, b2, b3, q0, q1);
                h[0][cc] = {a0.r + p0.r, a0.i + p0.i};
                h[1][cc] = {a1.r + p1.r, a1.i + p1.i};
                g[0][cc] = {b0.r - q0.r, b0.i - q0.i};
                g[1][cc] = {b1.r - q1.r, b1.i - q1.i};
            }
            for (int jj = 0; jj < 2; ++jj)
                for (int x = 0; x < 3; ++x)
                    for (int y = 0; y < 3; ++y) {
                        cplx t = cmulc(h[jj][x], g[jj][y]);
                        B[3 * x + y].r += sg * t.r;
                        B[3 * x + y].i += sg * t.i;
                    }
        }
    }
    const double2* Ul = U + ((size_t)mu * V + i) * 9;
    cplx u[9];
    for (int q = 0; q < 9; ++q) u[q] = {Ul[q].x, Ul[q].y};
    // W = sigma k (U B^dag - B U^dag);  Y = -i W
    cplx Y[9];
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            cplx w = {0.0, 0.0};
            for (int q = 0; q < 3; ++q) {
                cplx t1 = cmulc(u[3 * x + q], B[3 * y + q]);   // U_xq conj(B_yq)
                cplx t2 = cmulc(B[3 * x + q], u[3 * y + q]);   // B_xq conj(U_yq)
                w.r += t1.r - t2.r;
                w.i += t1.i - t2.i;
            }
            w.r *= sigma * k;
            w.i *= sigma * k;
            Y[3 * x + y] = {w.i, -w.r};
        }
    // F = 1/4 [ (Y + Y^dag)/2 - tr(Y + Y^dag)/6 ]
    const double tr = (Y[0].r + Y[4].r + Y[8].r) / 3.0;
    double2* Fl = F + ((size_t)mu * V + i) * 9;
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            const cplx a = Y[3 * x + y], b = Y[3 * y + x];
            double re = 0.5 * (a.r + b.r), im = 0.5 * (a.i - b.i);
            if (x == y) re -= tr;
            Fl[3 * x + y] = make_double2(0.25 * re, 0.25 * im);
        }
    if (G) {
        double2* Gl = G + ((size_t)mu * V + i) * 9;
        const double f = -sigma * k;
        for (int q = 0; q < 9; ++q) Gl[q] = make_double2(f * B[q].r, f * B[q].i);
    }
}

// ---------------------------------------------------------------------------
// MD: P <- P - dt_p F ; U <- exp(i dt_u P) U ; partial sum of tr P^2.
// exp by scaling and squaring of a degree-16 Taylor polynomial
// (argument norm <= 1/2 after scaling: truncation below 1e-19).
// ---------------------------------------------------------------------------
__device__ void mat3_mul(const cplx* a, const cplx* b, cplx* o) {
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            cplx t = {0.0, 0.0};
            for (int q = 0; q < 3; ++q) {
                cplx m = cmul(a[3 * x + q], b[3 * q + y]);
                t.r += m.r; t.i += m.i;
            }
            o[3 * x + y] = t;
        }
}

__global__ void __launch_bounds__(256) k_md_update(double2* __restrict__ U, double2* __restrict__ P,
                                                   const double2* __restrict__ F, double dt_p,
                                                   double dt_u, int nlink, double* partial) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    double kin = 0;
    if (l < nlink) {
        cplx p[9];
        for (int q = 0; q < 9; ++q) p[q] = {P[(size_t)l * 9 + q].x, P[(size_t)l * 9 + q].y};
        if (F && dt_p != 0.0) {
            for (int q = 0; q < 9; ++q) {
                p[q].r -= dt_p * F[(size_t)l * 9 + q].x;
                p[q].i -= dt_p * F[(size_t)l * 9 + q].y;
            }
            for (int q = 0; q < 9; ++q) P[(size_t)l * 9 + q] = make_double2(p[q].r, p[q].i);
        }
        if (dt_u != 0.0) {
            cplx X[9];   // X = i dt_u P
            double nrm = 0;
            for (int q = 0; q < 9; ++q) {
                X[q] = {-dt_u * p[q].i, dt_u * p[q].r};
                nrm += X[q].r * X[q].r + X[q].i * X[q].i;
            }
            nrm = sqrt(nrm);
            int sq = 0;
            while (nrm > 0.5 && sq < 40) { nrm *= 0.5; ++sq; }
            const double scale = ldexp(1.0, -sq);
            for (int q = 0; q < 9; ++q) { X[q].r *= scale; X[q].i *= scale; }
            cplx E[9], T[9], W[9];
            for (int q = 0; q < 9; ++q) { E[q] = {q % 4 == 0 ? 1.0 : 0.0, 0.0}; T[q] = E[q]; }
            for (int nn = 1; nn <= 16; ++nn) {
                mat3_mul(T, X, W);
                const double inv = 1.0 / nn;
                for (int q = 0; q < 9; ++q) { T[q] = {W[q].r * inv, W[q].i * inv}; E[q].r += T[q].r; E[q].i += T[q].i; }
            }
            for (int r = 0; r < sq; ++r) {
                mat3_mul(E, E, W);
                for (int q = 0; q < 9; ++q) E[q] = W[q];
            }
            cplx u[9];
            for (int q = 0; q < 9; ++q) u[q] = {U[(size_t)l * 9 + q].x, U[(size_t)l * 9 + q].y};
            mat3_mul(E, u, W);
            for (int q = 0; q < 9; ++q) U[(size_t)l * 9 + q] = make_double2(W[q].r, W[q].i);
        }
        // tr(P^2) = sum_xy P_xy P_yx
        for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y) kin += cmul(p[3 * x + y], p[3 * y + x]).r;
    }
    if (partial) {
        __shared__ double red[4];
        double x = kin;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

hipError_t launch_force(const void* U, const void* chiL, const void* chiR, double k, void* F, void* G,
                        const int L[4], int Ls, int aperiodic, hipStream_t st) {
    const int V = L[0] * L[1] * L[2] * L[3];
    const int n = 4 * V;
    hipLaunchKernelGGL(k_force, dim3((n + 255) / 256), dim3(256), 0, st, (const double2*)U,
                       (const double2*)chiL, (const double2*)chiR, k, (double2*)F, (double2*)G,
                       L[0], L[1], L[2], L[3], Ls, aperiodic);
    return hipGetLastError();
}

int md_blocks(int nlink) { return (nlink + 255) / 256; }

hipError_t launch_md_update(void* U, void* P, const void* F, double dt_p, double dt_u, int nlink,
                            double* partial, hipStream_t st) {
    hipLaunchKernelGGL(k_md_update, dim3(md_blocks(nlink)), dim3(256), 0, st, (double2*)U, (double2*)P,
                       (const double2*)F, dt_p, dt_u, nlink, partial);
    return hipGetLastError();
}

}  // namespace eofa
