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
// FP64 throughout; one work-item per 5D site, fields in the FP64 device layout.
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

// F and G of one link from B = B[chi_L] - B[chi_R] and the link U (natural
// layout entries, row major), sigma the boundary sign of the link:
//   W = sigma k (U B^dag - B U^dag),  F = 1/4 TA(-i W),  G = -sigma k B.
__device__ __forceinline__ void force_from_B(const cplx (&B)[9], const double2* __restrict__ Ul, double sigma, double k,
                             double2* __restrict__ Fl, double2* __restrict__ Gl) {
    cplx u[9];
    for (int q = 0; q < 9; ++q) u[q] = {Ul[q].x, Ul[q].y};
    cplx Y[9];   // Y = -i W
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            cplx w = {0.0, 0.0};
            for (int q = 0; q < 3; ++q) {
                const cplx t1 = cmulc(u[3 * x + q], B[3 * y + q]);   // U_xq conj(B_yq)
                const cplx t2 = cmulc(B[3 * x + q], u[3 * y + q]);   // B_xq conj(U_yq)
                w.r += t1.r - t2.r;
                w.i += t1.i - t2.i;
            }
            w.r *= sigma * k;
            w.i *= sigma * k;
            Y[3 * x + y] = {w.i, -w.r};
        }
    // F = 1/4 [ (Y + Y^dag)/2 - tr(Y + Y^dag)/6 ]
    const double tr = (Y[0].r + Y[4].r + Y[8].r) / 3.0;
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            const cplx a = Y[3 * x + y], b = Y[3 * y + x];
            double re = 0.5 * (a.r + b.r), im = 0.5 * (a.i - b.i);
            if (x == y) re -= tr;
            Fl[3 * x + y] = make_double2(0.25 * re, 0.25 * im);
        }
    if (Gl) {
        const double f = -sigma * k;
        for (int q = 0; q < 9; ++q) Gl[q] = make_double2(f * B[q].r, f * B[q].i);
    }
}

// Work-item (site, s) of parity p, workgroups of NS whole sites
// x Ls slices in the per-site FP64 traversal (site table, XCD ranges).
// chi_L, chi_R in the FP64 device layout (block c of 5D site n at
// base[c N + n], n = cb Ls + s).  For each system and direction mu every
// work-item forms its slice's term of
// B_mu(x) = sum_{s, j} h_j(x, s) (x) g_j(x+mu, Ls-1-s)^dag; the Ls terms of a
// site are summed in LDS in a fixed order (chi_R's sums subtracted from
// chi_L's), and 4 NS work-items then finish the links of the workgroup's sites.
__global__ void __launch_bounds__(256, 3) k_force_dev(const double2* __restrict__ chiLe,
                                                   const double2* __restrict__ chiLo,
                                                   const double2* __restrict__ chiRe,
                                                   const double2* __restrict__ chiRo,
                                                   const double2* __restrict__ U, const int* __restrict__ nbr,
                                                   const int* __restrict__ sites, double k,
                                                   double2* __restrict__ F, double2* __restrict__ G, Geo g,
                                                   int NS, size_t N) {
    extern __shared__ double red[];   // [NT][19] slice terms, then [4][NS][18] sums
    const int NT = blockDim.x, tid = threadIdx.x, Ls = g.Ls;
    const int sl = tid / Ls, s = tid - sl * Ls;
    // the two parities of a slot range run back to back on one XCD, so the
    // spinors one reads as neighbours are still in L2 when the other reads
    // them as its own sites
    const int lbp = xcd_block(gridDim.x);
    const int p = lbp & 1, lb = lbp >> 1;
    const int slot = lb * NS + sl;
    const int cb = sites ? sites[slot] : slot;
    const bool active = cb < g.Vh;
    const double2* ownL = p ? chiLo : chiLe;
    const double2* othL = p ? chiLe : chiLo;
    const double2* ownR = p ? chiRo : chiRe;
    const double2* othR = p ? chiRe : chiRo;
    double* sums = red + (size_t)NT * 19;
    const size_t na = (size_t)cb * Ls + s;
    // the forward neighbours' indices, loaded once and before any gather
    int nbf[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) nbf[mu] = active ? nbr[((size_t)p * 8 + mu) * g.Vh + cb] : 0;
    // chi_L then chi_R: the work-item's own spinor is loaded once per system
    // and kept in registers over the four directions
#pragma unroll 1
    for (int sys = 0; sys < 2; ++sys) {
        const double2* a = sys ? ownR : ownL;
        const double2* b = sys ? othR : othL;
        double2 own[12];
        for (int q = 0; q < 12; ++q) own[q] = active ? a[q * N + na] : make_double2(0.0, 0.0);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            cplx acc[9];
            for (int q = 0; q < 9; ++q) acc[q] = {0.0, 0.0};
            if (active) {
                const size_t nn = (size_t)nbf[mu] * Ls + (Ls - 1 - s);
                cplx h[2][3], gg[2][3];
                for (int cc = 0; cc < 3; ++cc) {
                    const double2 b0 = b[cc * N + nn], b1 = b[(3 + cc) * N + nn];
                    const double2 b2 = b[(6 + cc) * N + nn], b3 = b[(9 + cc) * N + nn];
                    cplx p0, p1, q0, q1;
                    amul(mu, {own[6 + cc].x, own[6 + cc].y}, {own[9 + cc].x, own[9 + cc].y}, p0, p1);
                    amul(mu, {b2.x, b2.y}, {b3.x, b3.y}, q0, q1);
                    h[0][cc] = {own[cc].x + p0.r, own[cc].y + p0.i};
                    h[1][cc] = {own[3 + cc].x + p1.r, own[3 + cc].y + p1.i};
                    gg[0][cc] = {b0.x - q0.r, b0.y - q0.i};
                    gg[1][cc] = {b1.x - q1.r, b1.y - q1.i};
                }
                for (int j = 0; j < 2; ++j)
                    for (int x = 0; x < 3; ++x)
                        for (int y = 0; y < 3; ++y) {
                            const cplx t = cmulc(h[j][x], gg[j][y]);
                            acc[3 * x + y].r += t.r;
                            acc[3 * x + y].i += t.i;
                        }
            }
            for (int q = 0; q < 9; ++q) {
                red[tid * 19 + 2 * q] = acc[q].r;
                red[tid * 19 + 2 * q + 1] = acc[q].i;
            }
            __syncthreads();
            // sum over s in a fixed order into sums[mu][site][18]: chi_L minus chi_R
            for (int t = tid; t < NS * 18; t += NT) {
                const int j = t / 18, q = t - 18 * j;
                double v = 0;
                for (int u = 0; u < Ls; ++u) v += red[(j * Ls + u) * 19 + q];
                double* dst = sums + mu * NS * 18 + t;
                *dst = sys ? *dst - v : v;
            }
            __syncthreads();
        }
    }
    // one work-item per (site, mu) finishes the links
    for (int t = tid; t < 4 * NS; t += NT) {
        const int mu = t / NS, j = t - mu * NS;
        const int slot2 = lb * NS + j;
        const int cb2 = sites ? sites[slot2] : slot2;
        if (cb2 >= g.Vh) continue;
        int c[4];
        const int i = natural_site(g, p, cb2, c);
        const double sigma = (mu == 3 && g.aperiodic && c[3] == g.L[3] - 1) ? -1.0 : 1.0;
        cplx B[9];
        const double* bs = sums + (mu * NS + j) * 18;
        for (int q = 0; q < 9; ++q) B[q] = {bs[2 * q], bs[2 * q + 1]};
        const size_t l = ((size_t)mu * g.V + i) * 9;
        force_from_B(B, U + l, sigma, k, F + l, G ? G + l : nullptr);
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

hipError_t launch_force(const void* U, const void* chiLe, const void* chiLo, const void* chiRe,
                        const void* chiRo, const int* nbr, const int* sites, double k, void* F, void* G,
                        const int L[4], int Ls, int aperiodic, int NS, int nblk, size_t N, hipStream_t st) {
    Geo g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = L[mu];
    g.V = L[0] * L[1] * L[2] * L[3];
    g.Vh = g.V / 2;
    g.Ls = Ls;
    g.aperiodic = aperiodic;
    const int NT = NS * Ls;
    const size_t shm = sizeof(double) * ((size_t)NT * 19 + (size_t)4 * NS * 18);
    hipLaunchKernelGGL(k_force_dev, dim3(2 * nblk), dim3(NT), shm, st, (const double2*)chiLe,
                       (const double2*)chiLo, (const double2*)chiRe, (const double2*)chiRo, (const double2*)U,
                       nbr, sites, k, (double2*)F, (double2*)G, g, NS, N);
    return hipGetLastError();
}

int md_blocks(int nlink) { return (nlink + 255) / 256; }

// Scratch of the allocation-free MD update: the per-block partial sums of
// tr P^2 that k_md_update writes and k_reduce adds up.  Each GPU holds its
// own copy for the life of the process.  In host code the name below is not
// a device address: the host reaches the array only through the pointer
// md_scratch_address returns (hipGetSymbolAddress on the current device).
static __device__ __align__(256) double scratch[MD_SCRATCH_DOUBLES];

hipError_t md_scratch_address(double** out) {
    return hipGetSymbolAddress((void**)out, HIP_SYMBOL(scratch));
}

hipError_t launch_md_update(void* U, void* P, const void* F, double dt_p, double dt_u, int nlink,
                            double* partial, hipStream_t st) {
    hipLaunchKernelGGL(k_md_update, dim3(md_blocks(nlink)), dim3(256), 0, st, (double2*)U, (double2*)P,
                       (const double2*)F, dt_p, dt_u, nlink, partial);
    return hipGetLastError();
}

}  // namespace eofa
