// gauge.hip -- gauge action of the ensembles (Table 1: Iwasaki) and its force.
//
//   S_g = beta sum_x [ c0 sum_{mu<nu} (1 - Re tr W_1x1/3) + c1 sum_{mu!=nu} (1 - Re tr W_2x1/3) ]
// with c0 = 1 - 8 c1; W_2x1 is the loop two links long in mu and one in nu.
// c1 = -0.331 is the Iwasaki action, c1 = 0 the Wilson action.  Links are
// periodic in every direction (the fermion boundary phase is not part of U).
//
// Force: S_g depends on one link U_mu(x) through -(beta/3) Re tr(U_mu(x) Sigma)
// with Sigma the weighted sum of the staples (the rest of every loop through
// the link, walked from x+mu back to x).  With Omega = U Sigma and the
// convention of the fermion force (F = sum_a T^a d^a S, d^a along
// U -> exp(i eps T^a) U, T^a = lambda^a/2):
//   F = -(beta/12) (Y - tr(Y)/3),  Y = i (Omega - Omega^dag).
// Per plane (mu, nu), nu != mu, a link sits in two plaquettes and six
// rectangles: four long in mu (the link first or second along mu, nu up or
// down) and two long in nu (nu up or down).  Staples that end in the same
// link share it, so the per-plane cost is 22 SU(3) products.
//
// FP64 throughout, natural gauge layout U[mu][i][3][3] (i the natural site
// index).  One work-item per link (force) or per site (action); blocks are
// mapped to contiguous ranges of links per XCD so that neighbouring links
// are shared within one L2.
#include "internal.h"

namespace eofa {

namespace {

struct M3 {
    double2 e[9];
};

__device__ __forceinline__ M3 ldm(const double2* __restrict__ U, size_t link) {
    M3 m;
    const double2* p = U + link * 9;
#pragma unroll
    for (int q = 0; q < 9; ++q) m.e[q] = p[q];
    return m;
}

// a b
__device__ __forceinline__ M3 mul_nn(const M3& a, const M3& b) {
    M3 o;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double2 u = a.e[3 * x + q], v = b.e[3 * q + y];
                re = fma(u.x, v.x, fma(-u.y, v.y, re));
                im = fma(u.x, v.y, fma(u.y, v.x, im));
            }
            o.e[3 * x + y] = make_double2(re, im);
        }
    return o;
}
// a b^dag
__device__ __forceinline__ M3 mul_nd(const M3& a, const M3& b) {
    M3 o;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {   // a_xq conj(b_yq)
                const double2 u = a.e[3 * x + q], v = b.e[3 * y + q];
                re = fma(u.x, v.x, fma(u.y, v.y, re));
                im = fma(u.y, v.x, fma(-u.x, v.y, im));
            }
            o.e[3 * x + y] = make_double2(re, im);
        }
    return o;
}
// a^dag b
__device__ __forceinline__ M3 mul_dn(const M3& a, const M3& b) {
    M3 o;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {   // conj(a_qx) b_qy
                const double2 u = a.e[3 * q + x], v = b.e[3 * q + y];
                re = fma(u.x, v.x, fma(u.y, v.y, re));
                im = fma(u.x, v.y, fma(-u.y, v.x, im));
            }
            o.e[3 * x + y] = make_double2(re, im);
        }
    return o;
}
__device__ __forceinline__ M3 dag(const M3& a) {
    M3 o;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) o.e[3 * x + y] = make_double2(a.e[3 * y + x].x, -a.e[3 * y + x].y);
    return o;
}
__device__ __forceinline__ M3 scaled(double s, const M3& a) {
    M3 o;
#pragma unroll
    for (int q = 0; q < 9; ++q) o.e[q] = make_double2(s * a.e[q].x, s * a.e[q].y);
    return o;
}
// o += s a
__device__ __forceinline__ void axpy(M3& o, double s, const M3& a) {
#pragma unroll
    for (int q = 0; q < 9; ++q) o.e[q] = make_double2(fma(s, a.e[q].x, o.e[q].x), fma(s, a.e[q].y, o.e[q].y));
}
// Re tr(a b^dag)
__device__ __forceinline__ double retr_nd(const M3& a, const M3& b) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) t = fma(a.e[q].x, b.e[q].x, fma(a.e[q].y, b.e[q].y, t));
    return t;
}

struct Lat {
    int L[4];
    int stride[4];
    int V;
};

__device__ __forceinline__ void coords(const Lat& g, int i, int (&c)[4]) {
    int r = i;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        c[d] = r % g.L[d];
        r /= g.L[d];
    }
}

// natural index of x + a e_mu + b e_nu (periodic) for |a|, |b| <= 2 and
// every extent >= 2: one wrap per direction suffices
__device__ __forceinline__ int shift2(const Lat& g, const int (&c)[4], int i, int mu, int a, int nu, int b) {
    int cm = c[mu] + a, cn = c[nu] + b;
    cm = cm < 0 ? cm + g.L[mu] : (cm >= g.L[mu] ? cm - g.L[mu] : cm);
    cn = cn < 0 ? cn + g.L[nu] : (cn >= g.L[nu] ? cn - g.L[nu] : cn);
    return i + (cm - c[mu]) * g.stride[mu] + (cn - c[nu]) * g.stride[nu];
}

}  // namespace

// One work-item per link l = mu V + i.
__global__ void __launch_bounds__(256) k_gauge_force(const double2* __restrict__ U, double2* __restrict__ F,
                                                     Lat g, double beta, double c1, int accumulate) {
    const int l = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    if (l >= 4 * g.V) return;
    const int mu = l / g.V, i = l - mu * g.V;
    const double c0 = 1.0 - 8.0 * c1;
    const bool rect = c1 != 0.0;
    int c[4];
    coords(g, i, c);
    const size_t V = (size_t)g.V;
    auto lk = [&](int d, int site) { return ldm(U, (size_t)d * V + site); };
    M3 sig;
#pragma unroll
    for (int q = 0; q < 9; ++q) sig.e[q] = make_double2(0.0, 0.0);
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        auto at = [&](int a, int b) { return shift2(g, c, i, mu, a, nu, b); };
        // loops above the link: every staple but the link-second rectangle
        // ends with U_nu(x)^dag
        const M3 B = mul_nd(lk(nu, at(1, 0)), lk(mu, at(0, 1)));          // U_nu(x+mu) U_mu(x+nu)^dag
        M3 T = scaled(c0, B);
        if (rect) {
            // U_mu(x+mu) U_nu(x+2mu) U_mu(x+mu+nu)^dag U_mu(x+nu)^dag
            M3 r = mul_nn(lk(mu, at(1, 0)), lk(nu, at(2, 0)));
            r = mul_nd(r, lk(mu, at(1, 1)));
            r = mul_nd(r, lk(mu, at(0, 1)));
            axpy(T, c1, r);
            // U_nu(x+mu) U_nu(x+mu+nu) U_mu(x+2nu)^dag U_nu(x+nu)^dag
            r = mul_nn(lk(nu, at(1, 0)), lk(nu, at(1, 1)));
            r = mul_nd(r, lk(mu, at(0, 2)));
            r = mul_nd(r, lk(nu, at(0, 1)));
            axpy(T, c1, r);
            // link second along mu: B U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
            r = mul_dn(lk(nu, at(-1, 0)), lk(mu, at(-1, 0)));
            r = mul_dn(lk(mu, at(-1, 1)), r);
            axpy(sig, c1, mul_nn(B, r));
        }
        axpy(sig, 1.0, mul_nd(T, lk(nu, i)));
        // loops below the link: every staple but the link-second rectangle
        // ends with U_nu(x-nu)
        const M3 D = dag(mul_nn(lk(mu, at(0, -1)), lk(nu, at(1, -1))));   // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag
        M3 Td = scaled(c0, D);
        if (rect) {
            // U_mu(x+mu) U_nu(x+2mu-nu)^dag U_mu(x+mu-nu)^dag U_mu(x-nu)^dag
            M3 r = mul_nn(lk(mu, at(0, -1)), lk(mu, at(1, -1)));
            r = mul_nn(r, lk(nu, at(2, -1)));
            axpy(Td, c1, mul_nd(lk(mu, at(1, 0)), r));
            // U_nu(x+mu-nu)^dag U_nu(x+mu-2nu)^dag U_mu(x-2nu)^dag U_nu(x-2nu)
            r = mul_nn(lk(mu, at(0, -2)), lk(nu, at(1, -2)));
            r = mul_nn(r, lk(nu, at(1, -1)));
            axpy(Td, c1, mul_dn(r, lk(nu, at(0, -2))));
            // link second along mu: D U_mu(x-mu-nu)^dag U_nu(x-mu-nu) U_mu(x-mu)
            r = mul_nn(lk(nu, at(-1, -1)), lk(mu, at(-1, 0)));
            r = mul_dn(lk(mu, at(-1, -1)), r);
            axpy(sig, c1, mul_nn(D, r));
        }
        axpy(sig, 1.0, mul_nn(Td, lk(nu, at(0, -1))));
    }
    // Omega = U Sigma; F = -(beta/12) (Y - tr Y / 3), Y = i (Omega - Omega^dag)
    const M3 Om = mul_nn(lk(mu, i), sig);
    const double f = -beta / 12.0;
    double trY = 0.0;
#pragma unroll
    for (int x = 0; x < 3; ++x) trY += -2.0 * Om.e[4 * x].y;
    double2* Fl = F + (size_t)l * 9;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const double2 a = Om.e[3 * x + y], b = Om.e[3 * y + x];
            // Y_xy = i (a - conj(b))
            double re = -(a.y + b.y), im = a.x - b.x;
            if (x == y) re -= trY / 3.0;
            double2 v = make_double2(f * re, f * im);
            if (accumulate) {
                const double2 o = Fl[3 * x + y];
                v.x += o.x;
                v.y += o.y;
            }
            Fl[3 * x + y] = v;
        }
}

// One work-item per site: c0 sum_{mu<nu} (1 - Re tr W_1x1/3) + c1 sum_{mu!=nu} (1 - Re tr W_2x1/3),
// summed per workgroup into partial[block].
__global__ void __launch_bounds__(256) k_gauge_action(const double2* __restrict__ U, Lat g, double c1,
                                                      double* __restrict__ partial) {
    const int i = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < g.V) {
        const double c0 = 1.0 - 8.0 * c1;
        const bool rect = c1 != 0.0;
        int c[4];
        coords(g, i, c);
        const size_t V = (size_t)g.V;
        auto lk = [&](int d, int site) { return ldm(U, (size_t)d * V + site); };
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
#pragma unroll 1
            for (int nu = 0; nu < 4; ++nu) {
                if (nu == mu) continue;
                auto at = [&](int a, int b) { return shift2(g, c, i, mu, a, nu, b); };
                const M3 um = lk(mu, i), un = lk(nu, i);
                if (mu < nu) {   // U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^dag
                    const double p = retr_nd(mul_nn(um, lk(nu, at(1, 0))), mul_nn(un, lk(mu, at(0, 1))));
                    acc = fma(c0, 1.0 - p / 3.0, acc);
                }
                if (rect) {      // U_mu(x) U_mu(x+mu) U_nu(x+2mu) [U_nu(x) U_mu(x+nu) U_mu(x+mu+nu)]^dag
                    const M3 a = mul_nn(mul_nn(um, lk(mu, at(1, 0))), lk(nu, at(2, 0)));
                    const M3 b = mul_nn(mul_nn(un, lk(mu, at(0, 1))), lk(mu, at(1, 1)));
                    acc = fma(c1, 1.0 - retr_nd(a, b) / 3.0, acc);
                }
            }
        }
    }
    __shared__ double red[4];
    double x = acc;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

static Lat make_lat(const int L[4]) {
    Lat g;
    int s = 1;
    for (int d = 0; d < 4; ++d) {
        g.L[d] = L[d];
        g.stride[d] = s;
        s *= L[d];
    }
    g.V = s;
    return g;
}

int gauge_force_blocks(int V) { return (4 * V + 255) / 256; }
int gauge_action_blocks(int V) { return (V + 255) / 256; }

hipError_t launch_gauge_force(const void* U, void* F, const int L[4], double beta, double c1, int accumulate,
                              hipStream_t st) {
    const Lat g = make_lat(L);
    hipLaunchKernelGGL(k_gauge_force, dim3(gauge_force_blocks(g.V)), dim3(256), 0, st, (const double2*)U,
                       (double2*)F, g, beta, c1, accumulate);
    return hipGetLastError();
}

hipError_t launch_gauge_action(const void* U, const int L[4], double c1, double* partial, hipStream_t st) {
    const Lat g = make_lat(L);
    hipLaunchKernelGGL(k_gauge_action, dim3(gauge_action_blocks(g.V)), dim3(256), 0, st, (const double2*)U, g, c1,
                       partial);
    return hipGetLastError();
}

}  // namespace eofa
