// dslash.hip -- the 5D Moebius domain-wall hopping kernel for gfx950.
//
// One work-item per 5D site (cb, s); a workgroup holds NS whole 4D sites
// times all Ls slices (NS*Ls work-items), so every operation that couples
// the fifth dimension stays inside the workgroup:
//
//   out = C( ch * A(Dh in) + ca * B(aux) + cr * aux2 )
//
// Dh is the Wilson hopping term of D_w (eq. (2.3)) between checkerboards,
// Dh = -1/2 sum_mu [(1-gamma_mu) U_mu(x) T+mu + (1+gamma_mu) U_mu(x-mu)^dag T-mu]
// (with the -1/2 and the boundary signs folded into the stored links), and
// its adjoint gamma_5 Dh gamma_5 when DAG.  The 4D site's links are shared
// by its Ls work-items, which read the same addresses.  A, B, C are the
// gauge-independent 5D operators of the Moebius/Cayley form (Section 2 and
// the Section 5.1 even-odd factorisation): Dtilde = b5 + c5 L,
// M_ee = (4-M5) Dtilde + 1 - L and M_ee^-1, with L or L^T.  Inverses use a
// weighted Hillis-Steele scan over s in LDS plus a rank-one wrap correction.
// The stencil is bandwidth-bound: no matrix cores.
#include "internal.h"

namespace eofa {

// ---------------------------------------------------------------------------
// spin projection in the chiral basis, gamma_mu = [[0, A_mu],[A_mu^dag, 0]],
// A_x = -i sigma_x, A_y = -i sigma_y, A_z = -i sigma_z, A_t = 1.
// (1 + sg gamma_mu) psi = (h ; sg A^dag h),  h = psi_up + sg A psi_lo.
// ---------------------------------------------------------------------------
template <int MU, int SG, typename A>
__device__ __forceinline__ void project(const A (&p)[24], A (&h)[12]) {
    // complex (spin k, colour c): re = p[2*(3k+c)], im = +1
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const A r0 = p[2 * c], i0 = p[2 * c + 1];
        const A r1 = p[2 * (3 + c)], i1 = p[2 * (3 + c) + 1];
        const A r2 = p[2 * (6 + c)], i2 = p[2 * (6 + c) + 1];
        const A r3 = p[2 * (9 + c)], i3 = p[2 * (9 + c) + 1];
        if constexpr (MU == 0) {        // A psi_lo = (-i psi3, -i psi2)
            h[2 * c] = r0 + SG * i3;       h[2 * c + 1] = i0 - SG * r3;
            h[6 + 2 * c] = r1 + SG * i2;   h[6 + 2 * c + 1] = i1 - SG * r2;
        } else if constexpr (MU == 1) { // A psi_lo = (-psi3, psi2)
            h[2 * c] = r0 - SG * r3;       h[2 * c + 1] = i0 - SG * i3;
            h[6 + 2 * c] = r1 + SG * r2;   h[6 + 2 * c + 1] = i1 + SG * i2;
        } else if constexpr (MU == 2) { // A psi_lo = (-i psi2, i psi3)
            h[2 * c] = r0 + SG * i2;       h[2 * c + 1] = i0 - SG * r2;
            h[6 + 2 * c] = r1 - SG * i3;   h[6 + 2 * c + 1] = i1 + SG * r3;
        } else {                        // A psi_lo = (psi2, psi3)
            h[2 * c] = r0 + SG * r2;       h[2 * c + 1] = i0 + SG * i2;
            h[6 + 2 * c] = r1 + SG * r3;   h[6 + 2 * c + 1] = i1 + SG * i3;
        }
    }
}

// acc_up += u ; acc_lo += sg A^dag u
template <int MU, int SG, typename A>
__device__ __forceinline__ void reconstruct(const A (&u)[12], A (&acc)[24]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const A r0 = u[2 * c], i0 = u[2 * c + 1];
        const A r1 = u[6 + 2 * c], i1 = u[6 + 2 * c + 1];
        acc[2 * c] += r0;           acc[2 * c + 1] += i0;
        acc[2 * (3 + c)] += r1;     acc[2 * (3 + c) + 1] += i1;
        A* l2 = &acc[2 * (6 + c)];
        A* l3 = &acc[2 * (9 + c)];
        if constexpr (MU == 0) {        // A^dag u = (i u1, i u0)
            l2[0] -= SG * i1; l2[1] += SG * r1;
            l3[0] -= SG * i0; l3[1] += SG * r0;
        } else if constexpr (MU == 1) { // A^dag u = (u1, -u0)
            l2[0] += SG * r1; l2[1] += SG * i1;
            l3[0] -= SG * r0; l3[1] -= SG * i0;
        } else if constexpr (MU == 2) { // A^dag u = (i u0, -i u1)
            l2[0] -= SG * i0; l2[1] += SG * r0;
            l3[0] += SG * i1; l3[1] -= SG * r1;
        } else {                        // A^dag u = (u0, u1)
            l2[0] += SG * r0; l2[1] += SG * i0;
            l3[0] += SG * r1; l3[1] += SG * i1;
        }
    }
}

// u(spin j) = link * h(spin j), link row major 3x3 complex; written as
// explicit fused multiply-add chains (two FMAs per real term)
template <typename A>
__device__ __forceinline__ void su3_mul(const A (&U)[18], const A (&h)[12], A (&u)[12]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const A* hj = &h[6 * j];
            const A* Ua = &U[6 * a];
            A re = Ua[0] * hj[0];
            A im = Ua[0] * hj[1];
            re = fmadd(-Ua[1], hj[1], re);
            im = fmadd(Ua[1], hj[0], im);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                re = fmadd(Ua[2 * b], hj[2 * b], re);
                re = fmadd(-Ua[2 * b + 1], hj[2 * b + 1], re);
                im = fmadd(Ua[2 * b], hj[2 * b + 1], im);
                im = fmadd(Ua[2 * b + 1], hj[2 * b], im);
            }
            u[6 * j + 2 * a] = re;
            u[6 * j + 2 * a + 1] = im;
        }
}

template <int P, bool DAG, int D>
__device__ __forceinline__ void hop_dir(const HopArgs& a, int site, int s,
                                        typename PT<P>::A (&acc)[24]) {
    using A = typename PT<P>::A;
    constexpr int MU = D & 3;
    constexpr int SG = (D < 4 ? -1 : 1) * (DAG ? -1 : 1);
    const int nb = a.nbr[(size_t)D * a.Vh + site];
    A psi[24];
    A h[12];
    if constexpr (P == P16 || P == PB16) {
        const float sc = ld_spinor_raw<P>(a.in, a.in_nrm, a.N, (size_t)nb * a.Ls + s, psi);
        project<MU, SG>(psi, h);
        if constexpr (P == P16) {
#pragma unroll
            for (int k = 0; k < 12; ++k) h[k] *= sc;
        }
    } else {
        ld_spinor<P>(a.in, a.in_nrm, a.N, (size_t)nb * a.Ls + s, psi);
        project<MU, SG>(psi, h);
    }
    A U[18];
    ld_link<P>(a.gauge, D, site, a.Vh, U);
    A u[12];
    su3_mul(U, h, u);
    reconstruct<MU, SG>(u, acc);
}

// ---------------------------------------------------------------------------
// 5D-local operators through LDS.  lds is [24][NT]; lane tid = sl*Ls + s.
// Shift S = L: upper spins (P+) shift down (s-1, wrap -m+), lower spins
// (P-) shift up (s+1, wrap -m-).  S = L^T: the directions swap.
// ---------------------------------------------------------------------------
template <typename A>
__device__ __forceinline__ void lds_put(A* lds, int NT, int tid, const A (&v)[24]) {
#pragma unroll
    for (int k = 0; k < 24; ++k) lds[k * NT + tid] = v[k];
}

template <typename A>
__device__ void op_bidiag_lds(A* lds, int NT, int tid, int s, int Ls, A (&v)[24],
                              const Op5& op, A mp, A mm) {
    lds_put(lds, NT, tid, v);
    __syncthreads();
    const int tdn = (s == 0) ? tid + Ls - 1 : tid - 1;
    const int tup = (s == Ls - 1) ? tid - (Ls - 1) : tid + 1;
    const bool up_down = !op.tr;   // upper chirality shifts down for L
    const int tu = up_down ? tdn : tup;
    const int tl = up_down ? tup : tdn;
    const A fu = (up_down ? s == 0 : s == Ls - 1) ? -mp : A(1);
    const A fl = (up_down ? s == Ls - 1 : s == 0) ? -mm : A(1);
    const A ca = (A)op.a, cb = (A)op.b;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = ca * v[k] + cb * fu * lds[k * NT + tu];
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] = ca * v[k] + cb * fl * lds[k * NT + tl];
    __syncthreads();
}

template <typename A>
__device__ __forceinline__ A ipow(A x, int e) {
    A r = 1;
    while (e > 0) { if (e & 1) r *= x; x *= x; e >>= 1; }
    return r;
}

// v <- (a + b S)^-1 v.  Along the shift direction (position q = s for a
// down shift, q = Ls-1-s for an up shift) the solution is
//   z_q = (1/a) sum_{j<=q} w^j v_{q-j},  w = -b/a   (scan)
//   y_q = z_q - m w^(q+1) z_last / (1 + m w^Ls)    (wrap-around term)
template <typename A>
__device__ void op_inverse_lds(A* lds, int NT, int tid, int s, int Ls, A (&v)[24],
                               const Op5& op, A mp, A mm) {
    const A ia = A(1) / (A)op.a;
    const A w = -(A)op.b * ia;
    const bool up_down = !op.tr;
    const int qu = up_down ? s : Ls - 1 - s;
    const int ql = up_down ? Ls - 1 - s : s;
    const int du = up_down ? -1 : 1;   // partner offset direction for upper comps
    const int dl = -du;
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] *= ia;
    A wd = w;
    for (int d = 1; d < Ls; d <<= 1) {
        lds_put(lds, NT, tid, v);
        __syncthreads();
        if (qu >= d) {
            const int t = tid + du * d;
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] += wd * lds[k * NT + t];
        }
        if (ql >= d) {
            const int t = tid + dl * d;
#pragma unroll
            for (int k = 12; k < 24; ++k) v[k] += wd * lds[k * NT + t];
        }
        __syncthreads();
        wd *= wd;
    }
    lds_put(lds, NT, tid, v);
    __syncthreads();
    const int base = tid - s;
    const int lu = up_down ? base + Ls - 1 : base;
    const int ll = up_down ? base : base + Ls - 1;
    const A wL = ipow(w, Ls);
    const A cu = -mp * ipow(w, qu + 1) / (A(1) + mp * wL);
    const A cl = -mm * ipow(w, ql + 1) / (A(1) + mm * wL);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] += cu * lds[k * NT + lu];
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] += cl * lds[k * NT + ll];
    __syncthreads();
}

template <typename A>
__device__ __forceinline__ void apply_op_lds(A* lds, int NT, int tid, int s, int Ls, A (&v)[24],
                                             const Op5& op, A mp, A mm) {
    if (op.kind == 1) op_bidiag_lds(lds, NT, tid, s, Ls, v, op, mp, mm);
    else if (op.kind == 2) op_inverse_lds(lds, NT, tid, s, Ls, v, op, mp, mm);
}

// double-precision workgroup sum; result valid in thread 0
__device__ __forceinline__ double block_sum(double x, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = x;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += red[i];
    }
    return t;
}

template <int P, bool DAG, bool HOP>
__global__ void __launch_bounds__(256, 3) k_hop(const HopArgs a) {
    using A = typename PT<P>::A;
    extern __shared__ unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    __shared__ double red[16];
    const int NT = blockDim.x;
    const int tid = threadIdx.x;
    const int Ls = a.Ls;
    const int sl = tid / Ls;
    const int s = tid - sl * Ls;
    const int lb = xcd_block(gridDim.x);
    const int site = (a.order ? a.order[lb] : lb) * a.NS + sl;
    const bool active = site < a.Vh;
    const size_t n = (size_t)site * Ls + s;
    const A mp = (A)a.mp, mm = (A)a.mm;

    A v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    if (HOP) {
        if (active) {
            hop_dir<P, DAG, 0>(a, site, s, v);
            hop_dir<P, DAG, 1>(a, site, s, v);
            hop_dir<P, DAG, 2>(a, site, s, v);
            hop_dir<P, DAG, 3>(a, site, s, v);
            hop_dir<P, DAG, 4>(a, site, s, v);
            hop_dir<P, DAG, 5>(a, site, s, v);
            hop_dir<P, DAG, 6>(a, site, s, v);
            hop_dir<P, DAG, 7>(a, site, s, v);
        }
        apply_op_lds(lds, NT, tid, s, Ls, v, a.opA, mp, mm);
        const A ch = (A)a.ch;
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] *= ch;
    }
    if (a.aux && active) {
        A x[24];
        ld_spinor<P>(a.aux, a.aux_nrm, a.N, n, x);
        const A ca = (A)a.ca;
        if (a.opB.kind == 1) {
            const bool up_down = !a.opB.tr;
            const size_t ndn = (s == 0) ? n + Ls - 1 : n - 1;
            const size_t nup = (s == Ls - 1) ? n - (Ls - 1) : n + 1;
            A xu[24], xl[24];
            ld_spinor<P>(a.aux, a.aux_nrm, a.N, up_down ? ndn : nup, xu);
            ld_spinor<P>(a.aux, a.aux_nrm, a.N, up_down ? nup : ndn, xl);
            const A fu = (up_down ? s == 0 : s == Ls - 1) ? -mp : A(1);
            const A fl = (up_down ? s == Ls - 1 : s == 0) ? -mm : A(1);
            const A ba = (A)a.opB.a, bb = (A)a.opB.b;
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] += ca * (ba * x[k] + bb * fu * xu[k]);
#pragma unroll
            for (int k = 12; k < 24; ++k) v[k] += ca * (ba * x[k] + bb * fl * xl[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] += ca * x[k];
        }
    }
    if (a.aux2 && active) {
        A x[24];
        ld_spinor<P>(a.aux2, a.aux2_nrm, a.N, n, x);
        const A cr = (A)a.cr;
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] += cr * x[k];
    }
    apply_op_lds(lds, NT, tid, s, Ls, v, a.opC, mp, mm);
    if (active) st_spinor<P>(a.out, a.out_nrm, a.N, n, v);
    if (a.partial) {
        double x = 0;
        if (active) {
#pragma unroll
            for (int k = 0; k < 24; ++k) x += (double)v[k] * (double)v[k];
        }
        x = block_sum(x, red);
        if (tid == 0) a.partial[blockIdx.x] = x;   // order-independent slot
    }
}

// ---------------------------------------------------------------------------
// CG search-direction update with the Cayley factor needed by the next
// Schur application:  p <- z + beta p  (beta = sc[i1]/sc[i0], or p <- z on
// the first call), pt <- Dtilde p = (b5 + c5 L) p.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_pupdate(const void* z, const float* z_nrm, void* p,
                                                 float* p_nrm, void* pt, float* pt_nrm,
                                                 const double* sc, int i_new, int i_old, int first,
                                                 int Vh, int Ls, int NS, size_t N, double b5,
                                                 double c5, double mp_, double mm_) {
    using A = typename PT<P>::A;
    extern __shared__ unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    const int NT = blockDim.x;
    const int tid = threadIdx.x;
    const int sl = tid / Ls;
    const int s = tid - sl * Ls;
    const int site = xcd_block(gridDim.x) * NS + sl;
    const bool active = site < Vh;
    const size_t n = (size_t)site * Ls + s;
    A v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    if (active) {
        ld_spinor<P>(z, z_nrm, N, n, v);
        if (!first) {
            const A beta = (A)(sc[i_new] / sc[i_old]);
            A q[24];
            ld_spinor<P>(p, p_nrm, N, n, q);
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] += beta * q[k];
        }
        st_spinor<P>(p, p_nrm, N, n, v);
    }
    Op5 op{1, 0, b5, c5};
    op_bidiag_lds(lds, NT, tid, s, Ls, v, op, (A)mp_, (A)mm_);
    if (active) st_spinor<P>(pt, pt_nrm, N, n, v);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int P, bool DAG, bool HOP>
static hipError_t launch_hop_t(const HopArgs& a, int nblk, hipStream_t st) {
    using A = typename PT<P>::A;
    const int NT = a.NS * a.Ls;
    const bool need_lds = (HOP && a.opA.kind != 0) || a.opC.kind != 0;
    const size_t shm = need_lds ? (size_t)24 * NT * sizeof(A) : 0;
    hipLaunchKernelGGL((k_hop<P, DAG, HOP>), dim3(nblk), dim3(NT), shm, st, a);
    return hipGetLastError();
}

hipError_t launch_hop(int prec, bool dag, bool hop, const HopArgs& a, int nblk, hipStream_t st) {
#define EOFA_CASE(PP)                                                         \
    case PP:                                                                  \
        if (hop) return dag ? launch_hop_t<PP, true, true>(a, nblk, st)       \
                            : launch_hop_t<PP, false, true>(a, nblk, st);     \
        return launch_hop_t<PP, false, false>(a, nblk, st);
    switch (prec) {
        EOFA_CASE(P64)
        EOFA_CASE(P32)
        EOFA_CASE(P16)
        EOFA_CASE(PB16)
    }
#undef EOFA_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_pupdate(int prec, const void* z, const float* zn, void* p, float* pn, void* pt,
                          float* ptn, const double* sc, int i_new, int i_old, int first, int Vh,
                          int Ls, int NS, size_t N, double b5, double c5, double mp, double mm,
                          int nblk, hipStream_t st) {
    const int NT = NS * Ls;
    switch (prec) {
#define EOFA_CASE(PP)                                                                         \
    case PP: {                                                                                \
        const size_t shm = (size_t)24 * NT * sizeof(typename PT<PP>::A);                      \
        hipLaunchKernelGGL((k_pupdate<PP>), dim3(nblk), dim3(NT), shm, st, z, zn, p, pn, pt,  \
                           ptn, sc, i_new, i_old, first, Vh, Ls, NS, N, b5, c5, mp, mm);      \
        return hipGetLastError();                                                             \
    }
        EOFA_CASE(P64)
        EOFA_CASE(P32)
        EOFA_CASE(P16)
        EOFA_CASE(PB16)
#undef EOFA_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace eofa
