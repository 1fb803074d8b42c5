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
// by its Ls work-items: the workgroup stages them in LDS once per launch.  A, B, C are the
// gauge-independent 5D operators of the Moebius/Cayley form (Section 2 and
// the Section 5.1 even-odd factorisation): Dtilde = b5 + c5 L,
// M_ee = (4-M5) Dtilde + 1 - L and M_ee^-1, with L or L^T.  Inverses use a
// weighted Hillis-Steele scan over s in LDS plus a rank-one wrap correction.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace eofa {

// ---------------------------------------------------------------------------
// spin projection in the chiral basis, gamma_mu = [[0, A_mu],[A_mu^dag, 0]],
// A_x = -i sigma_x, A_y = -i sigma_y, A_z = -i sigma_z, A_t = 1.
// (1 + sg gamma_mu) psi = (h ; sg A^dag h),  h = psi_up + sg A psi_lo.
// ---------------------------------------------------------------------------
template <int MU, typename A>
__device__ __forceinline__ void project(const A (&p)[24], A sg, A (&h)[12]) {
    // complex (spin k, colour c): re = p[2*(3k+c)], im = +1
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const A r0 = p[2 * c], i0 = p[2 * c + 1];
        const A r1 = p[2 * (3 + c)], i1 = p[2 * (3 + c) + 1];
        const A r2 = p[2 * (6 + c)], i2 = p[2 * (6 + c) + 1];
        const A r3 = p[2 * (9 + c)], i3 = p[2 * (9 + c) + 1];
        if constexpr (MU == 0) {        // A psi_lo = (-i psi3, -i psi2)
            h[2 * c] = r0 + sg * i3;       h[2 * c + 1] = i0 - sg * r3;
            h[6 + 2 * c] = r1 + sg * i2;   h[6 + 2 * c + 1] = i1 - sg * r2;
        } else if constexpr (MU == 1) { // A psi_lo = (-psi3, psi2)
            h[2 * c] = r0 - sg * r3;       h[2 * c + 1] = i0 - sg * i3;
            h[6 + 2 * c] = r1 + sg * r2;   h[6 + 2 * c + 1] = i1 + sg * i2;
        } else if constexpr (MU == 2) { // A psi_lo = (-i psi2, i psi3)
            h[2 * c] = r0 + sg * i2;       h[2 * c + 1] = i0 - sg * r2;
            h[6 + 2 * c] = r1 - sg * i3;   h[6 + 2 * c + 1] = i1 + sg * r3;
        } else {                        // A psi_lo = (psi2, psi3)
            h[2 * c] = r0 + sg * r2;       h[2 * c + 1] = i0 + sg * i2;
            h[6 + 2 * c] = r1 + sg * r3;   h[6 + 2 * c + 1] = i1 + sg * i3;
        }
    }
}

// acc_up += u ; acc_lo += sg A^dag u  (sg = +-1: a constant on the
// fixed-direction paths, per lane on the block paths)
template <int MU, typename A>
__device__ __forceinline__ void reconstruct(const A (&u)[12], A sg, A (&acc)[24]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const A r0 = u[2 * c], i0 = u[2 * c + 1];
        const A r1 = u[6 + 2 * c], i1 = u[6 + 2 * c + 1];
        acc[2 * c] += r0;           acc[2 * c + 1] += i0;
        acc[2 * (3 + c)] += r1;     acc[2 * (3 + c) + 1] += i1;
        A* l2 = &acc[2 * (6 + c)];
        A* l3 = &acc[2 * (9 + c)];
        if constexpr (MU == 0) {        // A^dag u = (i u1, i u0)
            l2[0] -= sg * i1; l2[1] += sg * r1;
            l3[0] -= sg * i0; l3[1] += sg * r0;
        } else if constexpr (MU == 1) { // A^dag u = (u1, -u0)
            l2[0] += sg * r1; l2[1] += sg * i1;
            l3[0] -= sg * r0; l3[1] -= sg * i0;
        } else if constexpr (MU == 2) { // A^dag u = (i u0, -i u1)
            l2[0] -= sg * i0; l2[1] += sg * r0;
            l3[0] += sg * i1; l3[1] -= sg * r1;
        } else {                        // A^dag u = (u0, u1)
            l2[0] += sg * r0; l2[1] += sg * i0;
            l3[0] += sg * r1; l3[1] += sg * i1;
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

// ---------------------------------------------------------------------------
// The links of the workgroup's NS sites are staged in LDS once per launch:
// the Ls work-items of a site then read them from LDS instead of each
// issuing the same global loads.  The staging loads are issued after the
// first neighbour-spinor loads so that both latencies overlap (FP64, whose
// registers hold one direction only, stages first and also keeps the
// neighbour indices in LDS).  Layout: [NS][8] link records of LB bytes,
// then [NS][8] neighbour indices (FP64),
//   P64      : 9 double2 (LB 144)
//   FP32 link: 9 float2, padded (LB 80) -- the FP32, BF16 and vector FP16 paths
//   MF       : 8 rows of 8 halves (LB 128), rows 6 and 7 zero (matrix cores)
// ---------------------------------------------------------------------------
template <int P, int MF> struct LinkLds {
    static constexpr int LB = MF ? 128 : (P == P64 ? 144 : 80);
};

__host__ __device__ constexpr size_t stage_bytes(int lb_bytes, int NS) {
    return (size_t)NS * 8 * lb_bytes + (size_t)NS * 8 * sizeof(int);
}

// Per-site paths (FP32 links for the vector paths, FP64 links for FP64):
// each slot's work-items stage their own slot's 72 link elements (q = 9 d + k)
// in batches of 4 per work-item, work-item (sl, s) taking q = s, s + Ls, ...;
// the site is the work-item's own, so no load waits on a table lookup.  FP64
// also stages the slot's 8 neighbour indices, placed after the links.
// Elements past the last repeat it (the same value to the same place).
template <int P>
__device__ __forceinline__ void stage_links(const HopArgs& a, int site, int sl, int s, unsigned char* lds) {
    constexpr int LB = LinkLds<P, 0>::LB;
    using T = typename std::conditional<P == P64, double2, float2>::type;
    const int Ls = a.Ls;
    if constexpr (P == P64) {
        int* nbl = reinterpret_cast<int*>(lds + (size_t)a.NS * 8 * LB) + sl * 8;
        for (int d = s; d < 8; d += Ls) nbl[d] = a.nbr[(size_t)d * a.Vh + site];
    }
    const size_t bb = (size_t)a.Vh * sizeof(T);
    const uint32_t off = (uint32_t)site * (uint32_t)sizeof(T);
    unsigned char* rec = lds + (size_t)sl * 8 * LB;
    for (int q0 = s; q0 < 72; q0 += 4 * Ls) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = at<T>(a.gauge, (size_t)min(q0 + u * Ls, 71) * bb, off);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = min(q0 + u * Ls, 71), d = q / 9, k = q - 9 * d;
            *reinterpret_cast<T*>(rec + d * LB + sizeof(T) * k) = v[u];
        }
    }
}

// The table-driven staging the dense (D_EOFA) hops keep: consecutive
// work-items take consecutive slots of one link element, looking each
// slot's site up in the traversal table.  Their kernels hold the dense
// blocks' LDS tile and measured faster with it (FP32: 114 against 154
// registers with the own-slot staging above).
__device__ __forceinline__ int slot_site(const HopArgs& a, int lb, int j) {
    const int slot = lb * a.NS + j;
    const int site = a.sites ? a.sites[slot] : slot;
    return site < a.Vh ? site : 0;   // padding slots read site 0 and discard it
}

template <int P>
__device__ __forceinline__ void stage_links_tbl(const HopArgs& a, int lb, unsigned char* lds) {
    constexpr int LB = LinkLds<P, 0>::LB;
    using T = typename std::conditional<P == P64, double2, float2>::type;
    const int NS = a.NS, NT = blockDim.x, tid = threadIdx.x;
    if constexpr (P == P64) {
        int* nbl = reinterpret_cast<int*>(lds + (size_t)NS * 8 * LB);
        for (int e = tid; e < NS * 8; e += NT) {
            const int j = e % NS, d = e / NS;
            nbl[j * 8 + d] = a.nbr[(size_t)d * a.Vh + slot_site(a, lb, j)];
        }
    }
    const size_t bb = (size_t)a.Vh * sizeof(T);
    for (int e = tid; e < NS * 72; e += NT) {
        const int j = e % NS, dk = e / NS;
        const int d = dk / 9, k = dk - 9 * d;
        *reinterpret_cast<T*>(lds + (j * 8 + d) * LB + sizeof(T) * k) =
            at<T>(a.gauge, (size_t)dk * bb, (uint32_t)slot_site(a, lb, j) * (uint32_t)sizeof(T));
    }
}

// The same staging for the block-sharing hops, from the block-major copy of
// the links (a.lnkb: the 64 records of a block contiguous, record (d, j) of
// 36 B compact 16-bit or 72 B FP32 links), so that a workgroup's link loads
// cover a few whole cache lines instead of one partial line per record.
// Consecutive work-items read consecutive words.  The staging has two parts:
// links_fetch issues the loads of a work-item's first LinkPre::K elements
// into registers, all at once and before the neighbour gathers, and
// links_put writes them to LDS, so that its writes wait for the links alone
// while the gathers stay in flight; elements beyond the first K (Ls < 16)
// are staged by links_put in further batches of K.
template <int P, int MF> struct LinkPre {
    static constexpr int K = 4;
    static constexpr int W = MF ? 3 : 2;   // 32-bit words per element
    static constexpr int E = MF ? 64 : 72; // elements per slot
    uint32_t w[K][W];
};

template <int P, int MF>
__device__ __forceinline__ void links_load(const HopArgs& a, int lb, int e0, LinkPre<P, MF>& pre) {
    using LP = LinkPre<P, MF>;
    const int NS = a.NS, NT = blockDim.x, last = NS * LP::E - 1;
    // first word of the workgroup's blocks: 64 records of 9 words (MF) or 9 word pairs
    const uint32_t* g = reinterpret_cast<const uint32_t*>(a.lnkb) + (size_t)lb * (NS >> 3) * 64 * 9 * (MF ? 1 : 2);
#pragma unroll
    for (int u = 0; u < LP::K; ++u) {
        // out-of-range elements (beyond the workgroup's records, or the zero
        // rows 6 and 7 of a matrix-core record) read a valid word and are
        // discarded by links_write
        const int e = min(e0 + u * NT, last);
        if constexpr (MF != 0) {
            const int r = e & 7, q = e >> 3;
            const uint32_t* w = g + (size_t)q * 9 + 3 * (min(r, 5) >> 1);
#pragma unroll
            for (int k = 0; k < 3; ++k) pre.w[u][k] = __builtin_nontemporal_load(w + k);   // read once per launch
        } else {
            const uint2 v = reinterpret_cast<const uint2*>(g)[e];
            pre.w[u][0] = v.x;
            pre.w[u][1] = v.y;
        }
    }
}

template <int P, int MF>
__device__ __forceinline__ void links_write(const HopArgs& a, int e0, const LinkPre<P, MF>& pre,
                                            unsigned char* lds) {
    using LP = LinkPre<P, MF>;
    constexpr int LB = LinkLds<P, MF>::LB;
    const int NS = a.NS, NT = blockDim.x, n = NS * LP::E;
    // work-items beyond the workgroup's records repeat the last element (the
    // value links_load fetched for it), so that every write is issued
    // unconditionally, which keeps the loads of links_fetch where they are
#pragma unroll
    for (int u = 0; u < LP::K; ++u) {
        const int ec = min(e0 + u * NT, n - 1);
        if constexpr (MF != 0) {
            // row r of the compact link's real 6x6 form, from 3 words of the
            // record (9 (re, im) half pairs): row 2a = (Ur_ab, -Ui_ab) for
            // b = 0..2, then 0; row 2a+1 = (Ui_ab, Ur_ab), then 0; rows 6, 7 zero
            const int r = ec & 7, q = ec >> 3;   // q = (block, d, slot) record index in the workgroup
            const int jj = q & 7, d = (q >> 3) & 7, j = ((q >> 6) << 3) + jj;
            const uint32_t w0 = pre.w[u][0], w1 = pre.w[u][1], w2 = pre.w[u][2];
            uint4 v = (r & 1) ? make_uint4(__builtin_amdgcn_alignbit(w0, w0, 16), __builtin_amdgcn_alignbit(w1, w1, 16),
                                           __builtin_amdgcn_alignbit(w2, w2, 16), 0u)
                              : make_uint4(w0 ^ 0x80000000u, w1 ^ 0x80000000u, w2 ^ 0x80000000u, 0u);
            if (r >= 6) v = make_uint4(0, 0, 0, 0);
            *reinterpret_cast<uint4*>(lds + (j * 8 + d) * LB + 16 * r) = v;
        } else {
            static_assert(P == P32, "the vector block path stages FP32 links (FP64: hop_blk_f64)");
            const int q = ec / 9, k = ec - 9 * q;
            const int jj = q & 7, d = (q >> 3) & 7, j = ((q >> 6) << 3) + jj;
            *reinterpret_cast<uint2*>(lds + (j * 8 + d) * LB + 8 * k) = make_uint2(pre.w[u][0], pre.w[u][1]);
        }
    }
}

template <int P, int MF>
__device__ __forceinline__ void links_fetch(const HopArgs& a, int lb, LinkPre<P, MF>& pre) {
    links_load<P, MF>(a, lb, threadIdx.x, pre);
}

template <int P, int MF>
__device__ __forceinline__ void links_put(const HopArgs& a, int lb, const LinkPre<P, MF>& pre, unsigned char* lds) {
    using LP = LinkPre<P, MF>;
    const int NT = blockDim.x;
    links_write<P, MF>(a, threadIdx.x, pre, lds);
#pragma unroll 1
    for (int e0 = threadIdx.x + LP::K * NT; e0 < a.NS * LP::E; e0 += LP::K * NT) {
        LinkPre<P, MF> more;
        links_load<P, MF>(a, lb, e0, more);
        links_write<P, MF>(a, e0, more, lds);
    }
}

// The same two-part staging for the per-site matrix-core path, by the
// slot's own work-items, whose site is known (no table lookup that would
// have to wait behind the gathers): work-item (sl, s) builds rows
// q = s, s + Ls, ... of its slot's 8 records (q = 8 d + r); rows past the
// last repeat it (a zero row).
template <int P>
__device__ __forceinline__ void links_load_site(const HopArgs& a, int site, int q0, LinkPre<P, 1>& pre) {
    const uint32_t* g = reinterpret_cast<const uint32_t*>(a.frag);
#pragma unroll
    for (int u = 0; u < LinkPre<P, 1>::K; ++u) {
        const int q = min(q0 + u * a.Ls, 63), d = q >> 3, r = q & 7;
        const uint32_t* w = g + ((size_t)d * a.Vh + site) * 9 + 3 * (min(r, 5) >> 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) pre.w[u][k] = __builtin_nontemporal_load(w + k);   // read once per launch
    }
}

template <int P>
__device__ __forceinline__ void links_write_site(const HopArgs& a, int sl, int q0, const LinkPre<P, 1>& pre,
                                                 unsigned char* lds) {
    constexpr int LB = LinkLds<P, 1>::LB;
#pragma unroll
    for (int u = 0; u < LinkPre<P, 1>::K; ++u) {
        const int q = min(q0 + u * a.Ls, 63), d = q >> 3, r = q & 7;   // row r as in links_write
        const uint32_t w0 = pre.w[u][0], w1 = pre.w[u][1], w2 = pre.w[u][2];
        uint4 v = (r & 1) ? make_uint4(__builtin_amdgcn_alignbit(w0, w0, 16), __builtin_amdgcn_alignbit(w1, w1, 16),
                                       __builtin_amdgcn_alignbit(w2, w2, 16), 0u)
                          : make_uint4(w0 ^ 0x80000000u, w1 ^ 0x80000000u, w2 ^ 0x80000000u, 0u);
        if (r >= 6) v = make_uint4(0, 0, 0, 0);
        *reinterpret_cast<uint4*>(lds + (sl * 8 + d) * LB + 16 * r) = v;
    }
}

template <int P>
__device__ __forceinline__ void links_put_site(const HopArgs& a, int site, int sl, int s, const LinkPre<P, 1>& pre,
                                               unsigned char* lds) {
    constexpr int K = LinkPre<P, 1>::K;
    links_write_site<P>(a, sl, s, pre, lds);
#pragma unroll 1
    for (int q0 = s + K * a.Ls; q0 < 64; q0 += K * a.Ls) {
        LinkPre<P, 1> more;
        links_load_site<P>(a, site, q0, more);
        links_write_site<P>(a, sl, q0, more, lds);
    }
}

// One direction's neighbour spinor, loaded ahead of its use.
template <int P> struct Stage {
    using A = typename PT<P>::A;
    A psi[24];    // neighbour spinor (16-bit fields: raw values, scale in nrm)
    float nrm;
};

// 5D index nb Ls + s of a neighbour's slice as a separate 32-bit multiply and
// add.  Fused into one 64-bit multiply-add, the unused high word of the
// addend may be given a register whose load is still in flight, and the
// gather then waits for every outstanding load.
__device__ __forceinline__ uint32_t slice5(int nb, int Ls, int s) {
    uint32_t m = (uint32_t)nb * (uint32_t)Ls;
    asm volatile("" : "+v"(m));
    return m + (uint32_t)s;
}

template <int P>
__device__ __forceinline__ void load_stage(const HopArgs& a, int s, int nb, Stage<P>& st, bool split = false) {
    const size_t n = split ? slice5(nb, a.Ls, s) : (size_t)nb * a.Ls + s;
    if constexpr (P == P16 || P == PB16) st.nrm = ld_spinor_raw<P>(a.in, a.in_nrm, a.N, n, st.psi);
    else ld_spinor<P>(a.in, a.in_nrm, a.N, n, st.psi);
}

// direction mu, projector sign sg = +-1 (per lane on the block paths)
template <int P, int MU>
__device__ __forceinline__ void compute_stage_sg(const Stage<P>& st, const unsigned char* lrec,
                                                 typename PT<P>::A sg, typename PT<P>::A (&acc)[24]) {
    using A = typename PT<P>::A;
    using L = typename PT<link_prec(P)>::A;
    const L* ul = reinterpret_cast<const L*>(lrec);
    A U[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) U[k] = (A)ul[k];
    A h[12];
    project<MU>(st.psi, sg, h);
    if constexpr (P == P16) {
#pragma unroll
        for (int k = 0; k < 12; ++k) h[k] *= st.nrm;
    }
    A u[12];
    su3_mul(U, h, u);
    reconstruct<MU>(u, sg, acc);
}

template <int P, bool DAG, int D>
__device__ __forceinline__ void compute_stage(const Stage<P>& st, const unsigned char* lrec,
                                              typename PT<P>::A (&acc)[24]) {
    using A = typename PT<P>::A;
    compute_stage_sg<P, D & 3>(st, lrec, (A)((D < 4 ? -1 : 1) * (DAG ? -1 : 1)), acc);
}

template <int P, bool DAG>
__device__ __forceinline__ void compute_stage_rt(const Stage<P>& st, int d, const unsigned char* lrec,
                                                 typename PT<P>::A (&acc)[24]) {
    switch (d) {   // d is a compile-time constant after unrolling
    case 0: compute_stage<P, DAG, 0>(st, lrec, acc); break;
    case 1: compute_stage<P, DAG, 1>(st, lrec, acc); break;
    case 2: compute_stage<P, DAG, 2>(st, lrec, acc); break;
    case 3: compute_stage<P, DAG, 3>(st, lrec, acc); break;
    case 4: compute_stage<P, DAG, 4>(st, lrec, acc); break;
    case 5: compute_stage<P, DAG, 5>(st, lrec, acc); break;
    case 6: compute_stage<P, DAG, 6>(st, lrec, acc); break;
    default: compute_stage<P, DAG, 7>(st, lrec, acc); break;
    }
}

// All eight directions: two neighbour spinors in flight (FP64: one, the
// registers allow no more), links from LDS.  Every work-item of the
// workgroup must call this (it contains the staging barrier); padding
// work-items pass site 0 and discard the result.
template <int P, bool DAG, bool DENSE>
__device__ __forceinline__ void hop_all(const HopArgs& a, int lb, unsigned char* lds, int site, int sl, int s,
                                        typename PT<P>::A (&acc)[24]) {
    constexpr int LB = LinkLds<P, 0>::LB;
    if constexpr (P == P64) {   // links and neighbour indices already staged by the caller
        const int* nbl = reinterpret_cast<const int*>(lds + (size_t)a.NS * 8 * LB) + sl * 8;
        const unsigned char* lr = lds + sl * 8 * LB;
        Stage<P> st;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            load_stage<P>(a, s, nbl[d], st);
            compute_stage_rt<P, DAG>(st, d, lr + d * LB, acc);
        }
        return;
    }
    constexpr int DEPTH = 2;
    int nb[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) nb[d] = a.nbr[(size_t)d * a.Vh + site];
    if constexpr (!DENSE) stage_links<P>(a, site, sl, s, lds);   // before the gathers: nothing to wait behind
    Stage<P> st[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) load_stage<P>(a, s, nb[d], st[d]);
    if constexpr (DENSE) stage_links_tbl<P>(a, lb, lds);
    __syncthreads();
    const unsigned char* lr = lds + sl * 8 * LB;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        compute_stage_rt<P, DAG>(st[d % DEPTH], d, lr + d * LB, acc);
        if (d + DEPTH < 8) load_stage<P>(a, s, nb[d + DEPTH], st[d % DEPTH]);
    }
}

// LDS bytes of the block paths' shared neighbour spinors, after the links:
// the matrix-core paths keep the raw 16-bit words ([3][NT] words of 16
// bytes, then [NT] FP16 site norms), the vector paths the spinor at the
// arithmetic precision ([24 sizeof(A) / 16][NT] words of 16 bytes)
__host__ __device__ constexpr size_t share_bytes(int P, bool mf, int NT) {
    return (size_t)NT * (mf ? 52 : (P == P64 ? 192 : 96));
}

// The block form of the vector paths: the workgroup holds whole
// 2x2x2x2 blocks, listed by the site table as for the matrix-core block path
// below (slot j = b_y + 2 b_z + 4 b_t, b_x = (b_y + b_z + b_t + parity) mod
// 2).  Along every direction mu one neighbour lies inside the block (+mu if
// b_mu = 0, -mu if b_mu = 1).  Each work-item loads its inside neighbour
// along x (the block's opposite-parity site in the same slot) and shares it
// through LDS, where the inside neighbours along y, z and t are those of
// slots j^1, j^2 and j^4; the four outside neighbours come from memory, two
// in flight.  5 gathers per work-item instead of 8.  Used for FP32 (FP64:
// hop_blk_f64, which stages its links in phases to keep 4 workgroups per CU).
template <int P, bool DAG>
__device__ __forceinline__ void hop_blk_vec(const HopArgs& a, int lb, unsigned char* lds, int sl, int s,
                                            typename PT<P>::A (&acc)[24]) {
    using A = typename PT<P>::A;
    constexpr int LB = LinkLds<P, 0>::LB;
    constexpr int CH = 24 * (int)sizeof(A) / 16;   // 16-byte words per spinor
    constexpr int K = 16 / (int)sizeof(A);          // reals per word
    const int tid = threadIdx.x, NT = blockDim.x;
    const int j = sl & 7;
    const int off = (j << 1) | ((__popc(j) + a.par) & 1);   // b_x + 2 b_y + 4 b_z + 8 b_t
    auto din = [&](int mu) { return mu + 4 * ((off >> mu) & 1); };
    auto sgn = [&](int d) { return (A)((d < 4 ? -1 : 1) * (DAG ? -1 : 1)); };
    // neighbour indices from the block-major table: x inside, then the outside ones
    const int* nb = a.nbrb + ((size_t)(lb * (a.NS >> 3) + (sl >> 3)) * 5) * 8 + j;
    uint4* sh = reinterpret_cast<uint4*>(lds + stage_bytes(LB, a.NS));
    auto put = [&](const Stage<P>& st) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            A w[K];
#pragma unroll
            for (int k = 0; k < K; ++k) w[k] = st.psi[K * c + k];
            sh[c * NT + tid] = __builtin_bit_cast(uint4, w);
        }
    };
    auto get = [&](int src, Stage<P>& st) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            struct W { A v[K]; };
            const W w = __builtin_bit_cast(W, sh[c * NT + src]);
#pragma unroll
            for (int k = 0; k < K; ++k) st.psi[K * c + k] = w.v[k];
        }
    };
    const unsigned char* lr = lds + sl * 8 * LB;
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    auto inside = [&](auto mu_c, Stage<P>& t) {   // inside neighbour along y, z or t, from LDS
        constexpr int MU = decltype(mu_c)::value;
        get((sl ^ (1 << (MU - 1))) * a.Ls + s, t);
        compute_stage_sg<P, MU>(t, lr + din(MU) * LB, sgn(din(MU)), acc);
    };
    auto outside = [&](auto mu_c, const Stage<P>& t) {
        constexpr int MU = decltype(mu_c)::value;
        const int d = din(MU) ^ 4;
        compute_stage_sg<P, MU>(t, lr + d * LB, sgn(d), acc);
    };
    int nbo[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) nbo[mu] = nb[8 * (mu + 1)];
    LinkPre<P, 0> pre;
    links_fetch<P, 0>(a, lb, pre);
    __builtin_amdgcn_sched_barrier(0);
    Stage<P> sx, o[2];
    load_stage<P>(a, s, nb[0], sx, true);
    load_stage<P>(a, s, nbo[0], o[0], true);
    load_stage<P>(a, s, nbo[1], o[1], true);
    __builtin_amdgcn_sched_barrier(0);
    links_put<P, 0>(a, lb, pre, lds);
    put(sx);
    __syncthreads();
    compute_stage_sg<P, 0>(sx, lr + din(0) * LB, sgn(din(0)), acc);
    outside(I0{}, o[0]);
    load_stage<P>(a, s, nbo[2], o[0], true);
    inside(I1{}, sx);
    outside(I1{}, o[1]);
    load_stage<P>(a, s, nbo[3], o[1], true);
    inside(I2{}, sx);
    outside(I2{}, o[0]);
    inside(I3{}, sx);
    outside(I3{}, o[1]);
}

// The FP64 block form.  Its shared spinors take 36.9 KB of LDS at 192
// work-items, so the links are staged one phase (two directions per site)
// at a time, 2.3 KB from the phase-ordered block-major copy, which keeps the
// workgroup within 40 KB: 4 workgroups per CU as in the per-site form.
// Phases: the inside x and y, the inside z and t (the shared spinors from
// LDS), the outside x and y, the outside z and t (from memory), each
// direction's operands one at a time (the registers hold one FP64 spinor
// besides the accumulator).  Requires 18 NS <= NS Ls, one link element
// per staging work-item.
template <bool DAG>
__device__ __forceinline__ void hop_blk_f64(const HopArgs& a, int lb, unsigned char* lds, int sl, int s,
                                            double (&acc)[24]) {
    constexpr int P = P64;
    constexpr int LB = LinkLds<P, 0>::LB;
    const int tid = threadIdx.x, NT = blockDim.x, NS = a.NS;
    const int j = sl & 7;
    const int off = (j << 1) | ((__popc(j) + a.par) & 1);   // b_x + 2 b_y + 4 b_z + 8 b_t
    // direction of phase ph, slot k: phases 0, 1 the inside directions of
    // mu = 2 (ph mod 2) + k, phases 2, 3 the outside ones
    auto dir = [&](int ph, int k) {
        const int mu = 2 * (ph & 1) + k;
        const int d = mu + 4 * ((off >> mu) & 1);
        return ph < 2 ? d : d ^ 4;
    };
    auto sgn = [](int d) { return (double)((d < 4 ? -1 : 1) * (DAG ? -1 : 1)); };
    const int* nb = a.nbrb + ((size_t)(lb * (NS >> 3) + (sl >> 3)) * 5) * 8 + j;
    uint4* sh = reinterpret_cast<uint4*>(lds);
    unsigned char* lk = lds + share_bytes(P, false, NT);   // [NS][2] records of the phase, then 1 spare
    // staging element of this work-item: complex eq of the record of slot ek
    // of site ej; work-items beyond the NS*18 elements fetch site 0's and
    // store to the spare record (a branch here would split the kernel's
    // register ranges)
    const bool stager = tid < NS * 18;
    const int ej = stager ? tid / 18 : 0, ek = (tid / 9) & 1, eq = tid % 9;
    const double2* lsrc = reinterpret_cast<const double2*>(a.lnkb) +
                          (((size_t)lb * (NS >> 3) + (ej >> 3)) * 64 + ek * 8 + (ej & 7)) * 9 + eq;
    const int erec = stager ? ej * 2 + ek : NS * 2;
    auto fetch = [&](int ph) { return lsrc[(size_t)ph * 16 * 9]; };
    auto store = [&](double2 v) { *reinterpret_cast<double2*>(lk + erec * LB + 16 * eq) = v; };
    auto share = [&](const Stage<P>& st) {
#pragma unroll
        for (int c = 0; c < 12; ++c)
            sh[c * NT + tid] = __builtin_bit_cast(uint4, make_double2(st.psi[2 * c], st.psi[2 * c + 1]));
    };
    auto get = [&](int src, Stage<P>& st) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 w = __builtin_bit_cast(double2, sh[c * NT + src]);
            st.psi[2 * c] = w.x;
            st.psi[2 * c + 1] = w.y;
        }
    };
    // each phase's link element is loaded one phase ahead, so that the
    // stores between the barriers do not wait for memory
    double2 lnext = fetch(0);
    auto next_phase = [&](int ph) {   // every work-item; the previous phase's records are read
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        store(lnext);
        if (ph < 3) lnext = fetch(ph + 1);
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    };
    const unsigned char* l0 = lk + sl * 2 * LB;
    const unsigned char* l1 = l0 + LB;
    // the outside neighbours' indices, loaded before the first barrier
    int nbo[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) nbo[mu] = nb[8 * (mu + 1)];
    Stage<P> st;
    // phase 0: inside x (this work-item's load, shared) and inside y
    load_stage<P>(a, s, nb[0], st);
    store(lnext);
    lnext = fetch(1);
    share(st);
    __syncthreads();
    compute_stage_sg<P, 0>(st, l0, sgn(dir(0, 0)), acc);
    __builtin_amdgcn_sched_barrier(0);
    get((sl ^ 1) * a.Ls + s, st);
    compute_stage_sg<P, 1>(st, l1, sgn(dir(0, 1)), acc);
    next_phase(1);   // inside z and t
    get((sl ^ 2) * a.Ls + s, st);
    compute_stage_sg<P, 2>(st, l0, sgn(dir(1, 0)), acc);
    __builtin_amdgcn_sched_barrier(0);
    get((sl ^ 4) * a.Ls + s, st);
    compute_stage_sg<P, 3>(st, l1, sgn(dir(1, 1)), acc);
    next_phase(2);   // outside x and y
    load_stage<P>(a, s, nbo[0], st);
    compute_stage_sg<P, 0>(st, l0, sgn(dir(2, 0)), acc);
    __builtin_amdgcn_sched_barrier(0);
    load_stage<P>(a, s, nbo[1], st);
    compute_stage_sg<P, 1>(st, l1, sgn(dir(2, 1)), acc);
    next_phase(3);   // outside z and t
    load_stage<P>(a, s, nbo[2], st);
    compute_stage_sg<P, 2>(st, l0, sgn(dir(3, 0)), acc);
    __builtin_amdgcn_sched_barrier(0);
    load_stage<P>(a, s, nbo[3], st);
    compute_stage_sg<P, 3>(st, l1, sgn(dir(3, 1)), acc);
}

// ---------------------------------------------------------------------------
// FP16 hop on the matrix cores.  For 4 | Ls the four lanes of every 4x4x4
// MFMA block (v_mfma_f32_4x4x4_16b_f16: 16 independent blocks per wave,
// lane 4b+j supplies column j of B and row j of A) belong to one 4D site, so
// the link is the shared A operand and each lane's projected half spinor is
// its own B column:  (U h)_real = Ureal . h_real with
//   Ureal rows (re0, im0, re1, im1, re2, im2), columns in the same order,
//   row re_a = [Ur_a0, -Ui_a0, Ur_a1, -Ui_a1, Ur_a2, -Ui_a2, 0, 0]
//   row im_a = [Ui_a0,  Ur_a0, Ui_a1,  Ur_a1, Ui_a2,  Ur_a2, 0, 0].
// Inputs are FP16 (the stored spinor and an FP16 copy of the link), the
// products accumulate in FP32.  The spin projection is one packed FP16 add
// per complex number; the site norm and the reconstruction are FP32 FMAs.
// ---------------------------------------------------------------------------
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ h2v as_h2(uint32_t w) { return __builtin_bit_cast(h2v, w); }
__device__ __forceinline__ h2v mul_i(h2v y) {   // i y
    h2v t = __builtin_shufflevector(y, y, 1, 0);
    t.x = -t.x;
    return t;
}
__device__ __forceinline__ h4v cat(h2v a, h2v b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3); }
__device__ __forceinline__ h4v h4_of(uint32_t a, uint32_t b) { return cat(as_h2(a), as_h2(b)); }

// h_j (j = 0, 1) for colours c = 0..2 from the raw words w[3k + c]; sg = +-1
// (a constant on the fixed-direction paths, per lane on the block path)
template <int MU>
__device__ __forceinline__ void project_h2(const uint32_t (&w)[12], _Float16 sg, h2v (&h)[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2v p0 = as_h2(w[c]), p1 = as_h2(w[3 + c]), p2 = as_h2(w[6 + c]), p3 = as_h2(w[9 + c]);
        if constexpr (MU == 0) {        // h0 = p0 - sg i p3, h1 = p1 - sg i p2
            h[c] = p0 - sg * mul_i(p3);  h[3 + c] = p1 - sg * mul_i(p2);
        } else if constexpr (MU == 1) { // h0 = p0 - sg p3,   h1 = p1 + sg p2
            h[c] = p0 - sg * p3;         h[3 + c] = p1 + sg * p2;
        } else if constexpr (MU == 2) { // h0 = p0 - sg i p2, h1 = p1 + sg i p3
            h[c] = p0 - sg * mul_i(p2);  h[3 + c] = p1 + sg * mul_i(p3);
        } else {                        // h0 = p0 + sg p2,   h1 = p1 + sg p3
            h[c] = p0 + sg * p2;         h[3 + c] = p1 + sg * p3;
        }
    }
}

// acc_up += f u ; acc_lo += g A^dag u with g = sg f  (FMAs)
template <int MU>
__device__ __forceinline__ void reconstruct_f(const float (&u)[12], float f, float g, float (&acc)[24]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float r0 = u[2 * c], i0 = u[2 * c + 1];
        const float r1 = u[6 + 2 * c], i1 = u[6 + 2 * c + 1];
        acc[2 * c] = fmadd(f, r0, acc[2 * c]);
        acc[2 * c + 1] = fmadd(f, i0, acc[2 * c + 1]);
        acc[2 * (3 + c)] = fmadd(f, r1, acc[2 * (3 + c)]);
        acc[2 * (3 + c) + 1] = fmadd(f, i1, acc[2 * (3 + c) + 1]);
        float* l2 = &acc[2 * (6 + c)];
        float* l3 = &acc[2 * (9 + c)];
        if constexpr (MU == 0) {
            l2[0] = fmadd(-g, i1, l2[0]); l2[1] = fmadd(g, r1, l2[1]);
            l3[0] = fmadd(-g, i0, l3[0]); l3[1] = fmadd(g, r0, l3[1]);
        } else if constexpr (MU == 1) {
            l2[0] = fmadd(g, r1, l2[0]);  l2[1] = fmadd(g, i1, l2[1]);
            l3[0] = fmadd(-g, r0, l3[0]); l3[1] = fmadd(-g, i0, l3[1]);
        } else if constexpr (MU == 2) {
            l2[0] = fmadd(-g, i0, l2[0]); l2[1] = fmadd(g, r0, l2[1]);
            l3[0] = fmadd(g, i1, l3[0]);  l3[1] = fmadd(-g, r1, l3[1]);
        } else {
            l2[0] = fmadd(g, r0, l2[0]);  l2[1] = fmadd(g, i0, l2[1]);
            l3[0] = fmadd(g, r1, l3[0]);  l3[1] = fmadd(g, i1, l3[1]);
        }
    }
}

struct MStage {
    uint32_t w[12];   // raw 16-bit neighbour spinor (word c = complex c as (re, im))
    float nrm;
};

template <int P>
__device__ __forceinline__ void load_mstage(const HopArgs& a, int s, int nb, MStage& st, bool split = false) {
    const uint32_t n = split ? slice5(nb, a.Ls, s) : (uint32_t)nb * a.Ls + s;
    const uint32_t off = n * 16u;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const uint4 t = at<uint4>(a.in, (size_t)b * a.N * 16, off);
        st.w[4 * b] = t.x; st.w[4 * b + 1] = t.y; st.w[4 * b + 2] = t.z; st.w[4 * b + 3] = t.w;
    }
    if constexpr (P == P16) st.nrm = a.in_nrm[n];
    else st.nrm = 1.0f;
}

// Direction mu, sign sg = +-1 of the projector (1 + sg gamma_mu); lrec: the
// staged link record of this direction (8 rows of 16 bytes)
template <int MU>
__device__ __forceinline__ void compute_mstage(const MStage& st, const unsigned char* lrec, int lane4, float sg,
                                               float (&acc)[24]) {
    h2v h[6];
    project_h2<MU>(st.w, (_Float16)sg, h);
    const uint4 r0 = *reinterpret_cast<const uint4*>(lrec + 16 * lane4);
    const uint4 r1 = *reinterpret_cast<const uint4*>(lrec + 64 + 16 * lane4);
    const h4v A00 = h4_of(r0.x, r0.y), A01 = h4_of(r0.z, r0.w);
    const h4v A10 = h4_of(r1.x, r1.y), A11 = h4_of(r1.z, r1.w);
    const h2v z2 = {(_Float16)0, (_Float16)0};
    float u[12];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const h4v B0 = cat(h[3 * j], h[3 * j + 1]);
        const h4v B1 = cat(h[3 * j + 2], z2);
        f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        c0 = __builtin_amdgcn_mfma_f32_4x4x4f16(A00, B0, c0, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_4x4x4f16(A01, B1, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x4f16(A10, B0, c1, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x4f16(A11, B1, c1, 0, 0, 0);
        u[6 * j + 0] = c0[0]; u[6 * j + 1] = c0[1]; u[6 * j + 2] = c0[2]; u[6 * j + 3] = c0[3];
        u[6 * j + 4] = c1[0]; u[6 * j + 5] = c1[1];
    }
    reconstruct_f<MU>(u, st.nrm, sg * st.nrm, acc);
}

// BF16 on the matrix cores: the spin projection runs in FP32 on the
// unpacked words and is rounded back to BF16 (v_cvt_pk_bf16_f32) for the B
// operand; links, MFMA layout and reconstruction are those of the FP16 path
// (BF16 fields carry no site norm).
typedef short s4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s4v s4_of(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(s4v, make_uint2(a, b));
}
__device__ __forceinline__ float b16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float b16hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack_b16(float re, float im) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)re) |
           ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)im) << 16);
}

// h_j (j = 0, 1) for colours c = 0..2 as packed (re, im) BF16 words, the
// same projection as project() on the stored words
template <int MU>
__device__ __forceinline__ void project_b16(const uint32_t (&w)[12], float sg, uint32_t (&h)[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float r0 = b16lo(w[c]), i0 = b16hi(w[c]), r1 = b16lo(w[3 + c]), i1 = b16hi(w[3 + c]);
        const float r2 = b16lo(w[6 + c]), i2 = b16hi(w[6 + c]), r3 = b16lo(w[9 + c]), i3 = b16hi(w[9 + c]);
        if constexpr (MU == 0) {
            h[c] = pack_b16(r0 + sg * i3, i0 - sg * r3);  h[3 + c] = pack_b16(r1 + sg * i2, i1 - sg * r2);
        } else if constexpr (MU == 1) {
            h[c] = pack_b16(r0 - sg * r3, i0 - sg * i3);  h[3 + c] = pack_b16(r1 + sg * r2, i1 + sg * i2);
        } else if constexpr (MU == 2) {
            h[c] = pack_b16(r0 + sg * i2, i0 - sg * r2);  h[3 + c] = pack_b16(r1 - sg * i3, i1 + sg * r3);
        } else {
            h[c] = pack_b16(r0 + sg * r2, i0 + sg * i2);  h[3 + c] = pack_b16(r1 + sg * r3, i1 + sg * i3);
        }
    }
}

template <int MU>
__device__ __forceinline__ void compute_mstage_b16(const MStage& st, const unsigned char* lrec, int lane4, float sg,
                                                   float (&acc)[24]) {
    uint32_t h[6];
    project_b16<MU>(st.w, sg, h);
    const uint4 r0 = *reinterpret_cast<const uint4*>(lrec + 16 * lane4);
    const uint4 r1 = *reinterpret_cast<const uint4*>(lrec + 64 + 16 * lane4);
    const s4v A00 = s4_of(r0.x, r0.y), A01 = s4_of(r0.z, r0.w);
    const s4v A10 = s4_of(r1.x, r1.y), A11 = s4_of(r1.z, r1.w);
    float u[12];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const s4v B0 = s4_of(h[3 * j], h[3 * j + 1]);
        const s4v B1 = s4_of(h[3 * j + 2], 0u);
        f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        c0 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A00, B0, c0, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A01, B1, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A10, B0, c1, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A11, B1, c1, 0, 0, 0);
        u[6 * j + 0] = c0[0]; u[6 * j + 1] = c0[1]; u[6 * j + 2] = c0[2]; u[6 * j + 3] = c0[3];
        u[6 * j + 4] = c1[0]; u[6 * j + 5] = c1[1];
    }
    reconstruct_f<MU>(u, 1.0f, sg, acc);
}

// direction mu with a per-lane projector sign
template <int P, int MU>
__device__ __forceinline__ void compute_mstage_sg(const MStage& st, const unsigned char* lrec, int lane4, float sg,
                                                  float (&acc)[24]) {
    if constexpr (P == P16) compute_mstage<MU>(st, lrec, lane4, sg, acc);
    else compute_mstage_b16<MU>(st, lrec, lane4, sg, acc);
}

template <int P, bool DAG>
__device__ __forceinline__ void compute_mstage_rt(const MStage& st, int d, const unsigned char* lrec, int lane4,
                                                  float (&acc)[24]) {
#define EOFA_MSTAGE(DD) \
    compute_mstage_sg<P, (DD) & 3>(st, lrec, lane4, (float)(((DD) < 4 ? -1 : 1) * (DAG ? -1 : 1)), acc);
    switch (d) {   // d is a compile-time constant after unrolling
    case 0: EOFA_MSTAGE(0) break;
    case 1: EOFA_MSTAGE(1) break;
    case 2: EOFA_MSTAGE(2) break;
    case 3: EOFA_MSTAGE(3) break;
    case 4: EOFA_MSTAGE(4) break;
    case 5: EOFA_MSTAGE(5) break;
    case 6: EOFA_MSTAGE(6) break;
    default: EOFA_MSTAGE(7) break;
    }
#undef EOFA_MSTAGE
}

// eight directions with DEPTH directions' neighbour spinors in flight;
// called by every work-item (staging barrier inside)
template <int P, bool DAG, int DEPTH>
__device__ __forceinline__ void hop_all_mfma(const HopArgs& a, int lb, unsigned char* lds, int site, int sl, int s,
                                             int lane4, float (&acc)[24]) {
    constexpr int LB = LinkLds<P, 1>::LB;
    int nb[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) nb[d] = a.nbr[(size_t)d * a.Vh + site];
    // the links first, written to LDS after the gathers are issued (as in
    // hop_blk_mfma)
    LinkPre<P, 1> pre;
    links_load_site<P>(a, site, s, pre);
    __builtin_amdgcn_sched_barrier(0);
    MStage st[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) load_mstage<P>(a, s, nb[d], st[d], true);
    __builtin_amdgcn_sched_barrier(0);
    links_put_site<P>(a, site, sl, s, pre, lds);
    __syncthreads();
    const unsigned char* lr = lds + sl * 8 * LB;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        compute_mstage_rt<P, DAG>(st[d % DEPTH], d, lr + d * LB, lane4, acc);
        if (d + DEPTH < 8) load_mstage<P>(a, s, nb[d + DEPTH], st[d % DEPTH]);
    }
}

// The same eight directions when the workgroup holds whole 2x2x2x2 blocks of
// the lattice (blocks at even coordinates; the site table lists the 8 sites
// of the output parity of each block, slot j = b_y + 2 b_z + 4 b_t with b the
// site's offsets in its block, and b_x = (b_y + b_z + b_t + parity) mod 2).
// Along every direction mu one neighbour of a site lies inside its block
// (+mu if b_mu = 0, -mu if b_mu = 1) and the other outside.  The inside
// neighbour along x is the block's opposite-parity site with the same slot
// j; each work-item loads that one (its slice s) and shares it through LDS,
// where the inside neighbours along y, z and t are those of slots j^1, j^2
// and j^4.  A work-item so gathers 5 neighbour spinors from memory instead
// of 8.  The projector signs depend on the site's offsets and are applied
// per lane.  Order: inside x, then outside and inside directions
// alternating, with two outside spinors in flight besides the one read from
// LDS (the register budget of the 5-wave FP16 kernel).
template <int P, bool DAG>
__device__ __forceinline__ void hop_blk_mfma(const HopArgs& a, int lb, unsigned char* lds, int sl, int s,
                                             int lane4, float (&acc)[24]) {
    constexpr int LB = LinkLds<P, 1>::LB;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int j = sl & 7;
    const int off = (j << 1) | ((__popc(j) + a.par) & 1);   // b_x + 2 b_y + 4 b_z + 8 b_t
    // inside direction of mu: mu (forward, projector sign -1) if b_mu = 0,
    // mu + 4 (backward, +1) if b_mu = 1; the outside direction is the other
    auto din = [&](int mu) { return mu + 4 * ((off >> mu) & 1); };
    auto sgn = [&](int d) { return (d < 4 ? -1.f : 1.f) * (DAG ? -1.f : 1.f); };
    // neighbour indices from the block-major table: x inside, then the outside ones
    const int* nb = a.nbrb + ((size_t)(lb * (a.NS >> 3) + (sl >> 3)) * 5) * 8 + j;
    const int nbx = nb[0];
    int nbo[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) nbo[mu] = nb[8 * (mu + 1)];
    LinkPre<P, 1> pre;
    links_fetch<P, 1>(a, lb, pre);
    __builtin_amdgcn_sched_barrier(0);
    MStage sx, o[2];
    load_mstage<P>(a, s, nbx, sx, true);
    load_mstage<P>(a, s, nbo[0], o[0], true);
    load_mstage<P>(a, s, nbo[1], o[1], true);
    __builtin_amdgcn_sched_barrier(0);
    links_put<P, 1>(a, lb, pre, lds);
    uint4* sh = reinterpret_cast<uint4*>(lds + stage_bytes(LB, a.NS));
    float* shn = reinterpret_cast<float*>(sh + 3 * NT);
#pragma unroll
    for (int b = 0; b < 3; ++b) sh[b * NT + tid] = make_uint4(sx.w[4 * b], sx.w[4 * b + 1], sx.w[4 * b + 2], sx.w[4 * b + 3]);
    if constexpr (P == P16) shn[tid] = sx.nrm;
    __syncthreads();
    const unsigned char* lr = lds + sl * 8 * LB;
    auto inside = [&](auto mu_c) {   // inside neighbour along y, z or t, from LDS
        constexpr int MU = decltype(mu_c)::value;
        const int src = (sl ^ (1 << (MU - 1))) * a.Ls + s;
        MStage t;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const uint4 q = sh[b * NT + src];
            t.w[4 * b] = q.x; t.w[4 * b + 1] = q.y; t.w[4 * b + 2] = q.z; t.w[4 * b + 3] = q.w;
        }
        t.nrm = P == P16 ? shn[src] : 1.0f;
        const int d = din(MU);
        compute_mstage_sg<P, MU>(t, lr + d * LB, lane4, sgn(d), acc);
    };
    auto outside = [&](auto mu_c, const MStage& st) {
        constexpr int MU = decltype(mu_c)::value;
        const int d = din(MU) ^ 4;
        compute_mstage_sg<P, MU>(st, lr + d * LB, lane4, sgn(d), acc);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    compute_mstage_sg<P, 0>(sx, lr + din(0) * LB, lane4, sgn(din(0)), acc);
    outside(I0{}, o[0]);
    load_mstage<P>(a, s, nbo[2], o[0], true);
    inside(I1{});
    outside(I1{}, o[1]);
    load_mstage<P>(a, s, nbo[3], o[1], true);
    inside(I2{});
    outside(I2{}, o[0]);
    inside(I3{});
    outside(I3{}, o[1]);
}

// ---------------------------------------------------------------------------
// 5D-local operators through LDS.  The tile holds one row of 24 reals per
// work-item (row tid = sl*Ls + s, odd stride STR so that column sweeps are
// free of bank conflicts).  A shift S = L moves the upper spins (P+) down
// (s-1, wrap -m+) and the lower spins (P-) up (s+1, wrap -m-); S = L^T
// swaps the directions.
//   row exchange : each work-item reads the shifted neighbour row (a + b S)
//   column sweep : work-item (sl, s) walks component c = s (+Ls, ...) of its
//                  site along the fifth dimension; bidiagonal ops take one
//                  pass and (a + b S)^-1 two: the recursion
//                  z_q = x_q / a + w z_{q-1} (w = -b/a, q the position along
//                  the shift) and the rank-one wrap-around correction
//                  y_q = z_q - m w^(q+1) z_last / (1 + m w^Ls).
// ---------------------------------------------------------------------------
constexpr int STR = 25;

template <typename A>
__device__ __forceinline__ void put_row(A* T, int tid, const A (&v)[24]) {
    A* r = T + tid * STR;
#pragma unroll
    for (int k = 0; k < 24; ++k) r[k] = v[k];
}
template <typename A>
__device__ __forceinline__ void get_row(const A* T, int tid, A (&v)[24]) {
    const A* r = T + tid * STR;
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = r[k];
}

// out = a x + b S x for the row x staged in T (all rows staged, synced)
template <typename A>
__device__ __forceinline__ void row_bidiag(const A* T, int tid, int s, int Ls, const A (&x)[24],
                                           A (&out)[24], A a, A b, int tr, A mp, A mm) {
    const int tdn = (s == 0) ? tid + Ls - 1 : tid - 1;
    const int tup = (s == Ls - 1) ? tid - (Ls - 1) : tid + 1;
    const bool up_down = !tr;
    const A* ru = T + (up_down ? tdn : tup) * STR;
    const A* rl = T + (up_down ? tup : tdn) * STR;
    const A fu = b * ((up_down ? s == 0 : s == Ls - 1) ? -mp : A(1));
    const A fl = b * ((up_down ? s == Ls - 1 : s == 0) ? -mm : A(1));
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = fmadd(fu, ru[k], a * x[k]);
#pragma unroll
    for (int k = 12; k < 24; ++k) out[k] = fmadd(fl, rl[k], a * x[k]);
}

// Dense 5D block (kind-3 Op5): v_s <- scale sum_t M[s][t] v_t, with M the
// P+ block for spins 0, 1 and the P- block for spins 2, 3.  The rows of the
// workgroup are staged in T; every work-item takes part (two barriers).
template <typename A>
__device__ void row_dense(A* T, int tid, int sl, int s, int Ls, A (&v)[24], const double* __restrict__ dm,
                          const Op5& op, A scale) {
    put_row(T, tid, v);
    __syncthreads();
    const double* Mu = dm + (size_t)(op.a != 0.0 ? 2 : 0) * Ls * Ls;
    const double* Ml = Mu + (size_t)Ls * Ls;
    const int rs = op.tr ? 1 : Ls, cs = op.tr ? Ls : 1;   // M[s][t] at s rs + t cs
    const A* base = T + sl * Ls * STR;
    A acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    for (int t = 0; t < Ls; ++t) {
        const A mu = (A)Mu[s * rs + t * cs], ml = (A)Ml[s * rs + t * cs];
        const A* r = base + t * STR;
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = fmadd(mu, r[k], acc[k]);
#pragma unroll
        for (int k = 12; k < 24; ++k) acc[k] = fmadd(ml, r[k], acc[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = scale * acc[k];
}

template <typename A>
__device__ __forceinline__ A ipow(A x, int e) {
    A r = 1;
    while (e > 0) { if (e & 1) r *= x; x *= x; e >>= 1; }
    return r;
}

// One in-order pass over a column: x_q <- f(x_q) for q = 0 .. Ls-1 at
// col[(s0 + ds q) STR], with f a (stateful) recursion step.  Loads are
// issued in batches of CB before the batch's stores, so a pass waits for the
// LDS latency once per batch rather than once per element (CB is set per
// precision by the registers it can spare).
template <int CB, typename A, typename F>
__device__ __forceinline__ void col_pass(A* col, int Ls, int s0, int ds, F&& f) {
    int q = 0;
    for (; q + CB <= Ls; q += CB) {
        A x[CB];
#pragma unroll
        for (int i = 0; i < CB; ++i) x[i] = col[(s0 + ds * (q + i)) * STR];
#pragma unroll
        for (int i = 0; i < CB; ++i) col[(s0 + ds * (q + i)) * STR] = f(x[i]);
    }
    for (; q < Ls; ++q) {
        const int id = (s0 + ds * q) * STR;
        col[id] = f(col[id]);
    }
}

// in-place column ops; element at position q along the shift is col[sq(q)*STR]
template <int CB, typename A>
__device__ void col_bidiag(A* col, int Ls, bool down, A a, A b, A m) {
    const int s0 = down ? 0 : Ls - 1, ds = down ? 1 : -1;
    A prev = -m * col[(s0 + ds * (Ls - 1)) * STR];
    col_pass<CB>(col, Ls, s0, ds, [&](A x) {
        const A y = fmadd(b, prev, a * x);
        prev = x;
        return y;
    });
}

// (a + b S)^-1 applied to xs times the column
template <int CB, typename A>
__device__ void col_inverse(A* col, int Ls, bool down, A a, A b, A m, A xs = A(1)) {
    const int s0 = down ? 0 : Ls - 1, ds = down ? 1 : -1;
    const A ia = A(1) / a, w = -b * ia, iax = ia * xs;
    A z = 0;
    col_pass<CB>(col, Ls, s0, ds, [&](A x) {
        z = fmadd(w, z, iax * x);
        return z;
    });
    const A K = -m * z / (A(1) + m * ipow(w, Ls));
    A pw = w;
    col_pass<CB>(col, Ls, s0, ds, [&](A x) {
        const A y = fmadd(K, pw, x);
        pw *= w;
        return y;
    });
}

// (a2 + b2 S)^-1 (a1 + b1 S) applied to the column in two passes instead of
// three: the bidiagonal op and the inverse's forward recursion run in one
// sweep (both walk the column in the same direction), then the inverse's
// rank-one wrap correction
template <int CB, typename A>
__device__ void col_bidiag_inverse(A* col, int Ls, bool down, A a1, A b1, A a2, A b2, A m) {
    const int s0 = down ? 0 : Ls - 1, ds = down ? 1 : -1;
    A prev = -m * col[(s0 + ds * (Ls - 1)) * STR];
    const A ia = A(1) / a2, w = -b2 * ia;
    A z = 0;
    col_pass<CB>(col, Ls, s0, ds, [&](A x) {
        const A y = fmadd(b1, prev, a1 * x);
        prev = x;
        z = fmadd(w, z, ia * y);
        return z;
    });
    const A K = -m * z / (A(1) + m * ipow(w, Ls));
    A pw = w;
    col_pass<CB>(col, Ls, s0, ds, [&](A x) {
        const A r = fmadd(K, pw, x);
        pw *= w;
        return r;
    });
}

template <int CB, typename A>
__device__ __forceinline__ void col_op(A* col, int Ls, bool upper, const Op5& op, A mp, A mm) {
    const bool down = upper != (op.tr != 0);
    const A m = upper ? mp : mm;
    if (op.kind == 1) col_bidiag<CB>(col, Ls, down, (A)op.a, (A)op.b, m);
    else if (op.kind == 2) col_inverse<CB>(col, Ls, down, (A)op.a, (A)op.b, m);
}

// v <- op2(scale * op1(v)) through a column sweep of the staged tile
template <int CB, typename A>
__device__ void column_phase(A* T, int tid, int sl, int s, int Ls, A (&v)[24], const Op5& op1,
                             A scale, const Op5& op2, A mp, A mm) {
    put_row(T, tid, v);
    __syncthreads();
    // the forms the solver uses take one or two passes per column: a
    // bidiagonal op and an inverse in the same direction are fused, and the
    // scale is folded into the coefficients (FP32 arithmetic only: in FP64
    // the fused sweep costs the hop two more spilled registers, and measured
    // slower)
    const int k1 = std::is_same<A, double>::value ? -1 : op1.kind, k2 = op2.kind;
    for (int c = s; c < 24; c += Ls) {
        A* col = T + sl * Ls * STR + c;
        const bool upper = c < 12;
        const A m = upper ? mp : mm;
        const bool d1 = upper != (op1.tr != 0), d2 = upper != (op2.tr != 0);
        if (k1 == 1 && k2 == 2 && d1 == d2) {
            col_bidiag_inverse<CB>(col, Ls, d1, scale * (A)op1.a, scale * (A)op1.b, (A)op2.a, (A)op2.b, m);
        } else if ((k1 == 1 && k2 == 0) || (k1 == 0 && k2 == 1)) {
            const Op5& o = k1 ? op1 : op2;
            col_bidiag<CB>(col, Ls, k1 ? d1 : d2, scale * (A)o.a, scale * (A)o.b, m);
        } else if ((k1 == 2 && k2 == 0) || (k1 == 0 && k2 == 2)) {
            const Op5& o = k1 ? op1 : op2;
            col_inverse<CB>(col, Ls, k1 ? d1 : d2, (A)o.a, (A)o.b, m, scale);
        } else {
            col_op<CB>(col, Ls, upper, op1, mp, mm);
            if (scale != A(1)) col_pass<CB>(col, Ls, 0, 1, [&](A x) { return x * scale; });
            col_op<CB>(col, Ls, upper, op2, mp, mm);
        }
    }
    __syncthreads();
    get_row(T, tid, v);
    __syncthreads();
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

template <int P, bool DAG, bool HOP, int MF, bool DENSE = false, bool BLK = false>
__global__ void __launch_bounds__(256, (MF == 3 && P == P16 && !DENSE) ? 5 : 3) k_hop(const HopArgs a) {
    using A = typename PT<P>::A;
    // column-sweep load batch: what each variant's register budget allows
    constexpr int COLB = P == P64 ? 1 : (P == P16 && MF) ? 4 : 8;
    extern __shared__ unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    __shared__ double red[16];
    const int tid = threadIdx.x;
    const int Ls = a.Ls;
    const int sl = tid / Ls;
    const int s = tid - sl * Ls;
    const int lb = xcd_block(gridDim.x);
    const int slot = lb * a.NS + sl;
    const int site = a.sites ? a.sites[slot] : slot;
    const bool active = site < a.Vh;
    const size_t n = (size_t)site * Ls + s;
    const A mp = (A)a.mp, mm = (A)a.mm;

    A v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    if (HOP) {
        // every work-item takes part (staging barrier; the MFMA needs the
        // whole wave); padding work-items read site 0 and discard it
        if constexpr (P == P64 && !BLK) {
            if constexpr (DENSE) stage_links_tbl<P>(a, lb, smem_raw);
            else stage_links<P>(a, active ? site : 0, sl, s, smem_raw);
            __syncthreads();
        }
        if constexpr (MF && BLK) hop_blk_mfma<P, DAG>(a, lb, smem_raw, sl, s, tid & 3, v);
        else if constexpr (MF) hop_all_mfma<P, DAG, MF>(a, lb, smem_raw, active ? site : 0, sl, s, tid & 3, v);
        else if constexpr (BLK && P == P64) hop_blk_f64<DAG>(a, lb, smem_raw, sl, s, v);
        else if constexpr (BLK) hop_blk_vec<P, DAG>(a, lb, smem_raw, sl, s, v);
        else if constexpr (P == P64) { if (active) hop_all<P, DAG, DENSE>(a, lb, smem_raw, site, sl, s, v); }
        else hop_all<P, DAG, DENSE>(a, lb, smem_raw, active ? site : 0, sl, s, v);
        if (!active) {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = 0;
        }
        __syncthreads();   // the epilogue reuses the staged LDS area
    }
    if constexpr (DENSE) {
        // D_EOFA's even-odd form: out = ch DA(hop) + ca DB(aux) + cr aux2
        // (local: out = ca DB(aux) + cr aux2), DA and DB dense or identity
        if (HOP) {
            if (a.opA.kind == 3) row_dense(lds, tid, sl, s, Ls, v, a.dmat, a.opA, (A)a.ch);
            else {
#pragma unroll
                for (int k = 0; k < 24; ++k) v[k] *= (A)a.ch;
            }
        }
        if (a.aux) {
            A x[24];
            if (active) ld_spinor<P, true>(a.aux, a.aux_nrm, a.N, n, x);
            else {
#pragma unroll
                for (int k = 0; k < 24; ++k) x[k] = 0;
            }
            if (a.opB.kind == 3) row_dense(lds, tid, sl, s, Ls, x, a.dmat, a.opB, (A)a.ca);
            else {
#pragma unroll
                for (int k = 0; k < 24; ++k) x[k] *= (A)a.ca;
            }
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] += x[k];
        }
        if (a.aux2 && active) {
            A x[24];
            ld_spinor<P, true>(a.aux2, a.aux2_nrm, a.N, n, x);
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = fmadd((A)a.cr, x[k], v[k]);
        }
    } else {
    double alpha = 1.0;
    if (a.dsc) {
        alpha = a.dsc[a.s_num] / a.dsc[a.s_den];
        if (a.s_alpha >= 0 && blockIdx.x == 0 && tid == 0) a.dsc[a.s_alpha] = alpha;
    }
    if (HOP) {
        A ch = (A)(a.ch * alpha);
        bool aux2_done = false;
        if (a.aux2 && a.opA.kind == 0) {   // fold cr * aux2 in before the 5D ops (A = 1)
            A x[24];
            if (active) ld_spinor<P, true>(a.aux2, a.aux2_nrm, a.N, n, x);
            else {
#pragma unroll
                for (int k = 0; k < 24; ++k) x[k] = 0;
            }
            const A cr = (A)a.cr;
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = fmadd(ch, v[k], cr * x[k]);
            ch = A(1);
            aux2_done = true;
        }
        if (a.opA.kind != 0 || a.opC.kind != 0) {
            column_phase<COLB>(lds, tid, sl, s, Ls, v, a.opA, ch, a.opC, mp, mm);
        } else if (ch != A(1)) {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] *= ch;
        }
        if (a.aux) {
            A x[24];
            if (active) ld_spinor<P, true>(a.aux, a.aux_nrm, a.N, n, x);
            else {
#pragma unroll
                for (int k = 0; k < 24; ++k) x[k] = 0;
            }
            const A ca = (A)(a.ca * alpha);
            if (a.opB2.kind != 0) {
                column_phase<COLB>(lds, tid, sl, s, Ls, x, a.opB, ca, a.opB2, mp, mm);
#pragma unroll
                for (int k = 0; k < 24; ++k) v[k] += x[k];
            } else if (a.opB.kind == 1) {
                put_row(lds, tid, x);
                __syncthreads();
                A bx[24];
                row_bidiag(lds, tid, s, Ls, x, bx, (A)a.opB.a, (A)a.opB.b, a.opB.tr, mp, mm);
#pragma unroll
                for (int k = 0; k < 24; ++k) v[k] = fmadd(ca, bx[k], v[k]);
                __syncthreads();
            } else {
#pragma unroll
                for (int k = 0; k < 24; ++k) v[k] = fmadd(ca, x[k], v[k]);
            }
        }
        if (a.aux2 && !aux2_done && active) {
            A x[24];
            ld_spinor<P, true>(a.aux2, a.aux2_nrm, a.N, n, x);
            const A cr = (A)a.cr;
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = fmadd(cr, x[k], v[k]);
        }
    } else {
        // local 5D operator: out = C(ca * B(aux)) + cr * aux2
        if (active) ld_spinor<P>(a.aux, a.aux_nrm, a.N, n, v);
        if (a.opB.kind != 0 || a.opC.kind != 0) {
            column_phase<COLB>(lds, tid, sl, s, Ls, v, a.opB, (A)(a.ca * alpha), a.opC, mp, mm);
        } else {
            const A ca = (A)(a.ca * alpha);
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] *= ca;
        }
        if (a.aux2 && active) {
            A x[24];
            ld_spinor<P, true>(a.aux2, a.aux2_nrm, a.N, n, x);
            const A cr = (A)a.cr;
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = fmadd(cr, x[k], v[k]);
        }
    }
    }   // !DENSE
    if (active) st_spinor<P, true>(a.out, a.out_nrm, a.N, n, v);
    if (a.partial) {
        double x = 0;
        if (active) {
            // per work-item sum in the arithmetic type, workgroup and global sums in FP64
            A q = 0;
#pragma unroll
            for (int k = 0; k < 24; ++k) q = fmadd(v[k], v[k], q);
            x = (double)q;
        }
        x = block_sum(x, red);
        if (tid == 0) a.partial[blockIdx.x] = x;   // order-independent slot
    }
}

// ---------------------------------------------------------------------------
// CG search-direction update with the Cayley factor needed by the next
// Schur application:  p <- z + beta p  (beta = sc[i1]/sc[i0], or p <- z on
// the first call), pt <- Dtilde p = (b5 + c5 L) p.  With pt == nullptr only
// the Cayley-transformed direction is kept: p <- Dtilde z + beta p.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_pupdate(const void* z, const float* z_nrm, const void* pold,
                                                 const float* pold_nrm, void* p,
                                                 float* p_nrm, void* pt, float* pt_nrm,
                                                 const double* sc, int i_new, int i_old, int first,
                                                 int Vh, int Ls, int NS, size_t N, double b5,
                                                 double c5, double mp_, double mm_) {
    using A = typename PT<P>::A;
    extern __shared__ unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    const int tid = threadIdx.x;
    const int sl = tid / Ls;
    const int s = tid - sl * Ls;
    const int site = xcd_block(gridDim.x) * NS + sl;
    const bool active = site < Vh;
    const size_t n = (size_t)site * Ls + s;
    A v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    if (!pt) {
        // search directions kept as pt = Dtilde p:  pt <- Dtilde z + beta pt_old
        if (active) ld_spinor<P>(z, z_nrm, N, n, v);
        put_row(lds, tid, v);
        __syncthreads();
        A t[24];
        row_bidiag(lds, tid, s, Ls, v, t, (A)b5, (A)c5, 0, (A)mp_, (A)mm_);
        if (active) {
            if (!first) {
                const A beta = (A)(sc[i_new] / sc[i_old]);
                A q[24];
                ld_spinor<P>(pold, pold_nrm, N, n, q);
#pragma unroll
                for (int k = 0; k < 24; ++k) t[k] = fmadd(beta, q[k], t[k]);
            }
            st_spinor<P>(p, p_nrm, N, n, t);
        }
        return;
    }
    if (active) {
        ld_spinor<P>(z, z_nrm, N, n, v);
        if (!first) {
            const A beta = (A)(sc[i_new] / sc[i_old]);
            A q[24];
            ld_spinor<P>(pold, pold_nrm, N, n, q);
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] += beta * q[k];
        }
        st_spinor<P>(p, p_nrm, N, n, v);
    }
    put_row(lds, tid, v);
    __syncthreads();
    A t[24];
    row_bidiag(lds, tid, s, Ls, v, t, (A)b5, (A)c5, 0, (A)mp_, (A)mm_);
    if (active) st_spinor<P>(pt, pt_nrm, N, n, t);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int P, bool DAG, bool HOP>
static hipError_t launch_hop_t(const HopArgs& a, int nblk, hipStream_t st) {
    using A = typename PT<P>::A;
    const int NT = a.NS * a.Ls;
    const bool need_lds = HOP ? (a.opA.kind != 0 || a.opC.kind != 0 || (a.aux && (a.opB.kind != 0 || a.opB2.kind != 0)))
                              : (a.opB.kind != 0 || a.opC.kind != 0);
    const size_t tile = need_lds ? (size_t)STR * NT * sizeof(A) : 0;
    if constexpr ((P == P16 || P == PB16) && HOP) {
        if (a.frag) {
            const size_t shm = std::max(tile, stage_bytes(LinkLds<P, 1>::LB, a.NS) + (a.blk ? share_bytes(P, true, NT) : 0));
            if (a.blk) {   // the block path keeps its own loads in flight
                hipLaunchKernelGGL((k_hop<P, DAG, HOP, 3, false, true>), dim3(nblk), dim3(NT), shm, st, a);
                return hipGetLastError();
            }
            if (a.depth >= 4) hipLaunchKernelGGL((k_hop<P, DAG, HOP, 4>), dim3(nblk), dim3(NT), shm, st, a);
            else if (a.depth == 3) hipLaunchKernelGGL((k_hop<P, DAG, HOP, 3>), dim3(nblk), dim3(NT), shm, st, a);
            else hipLaunchKernelGGL((k_hop<P, DAG, HOP, 2>), dim3(nblk), dim3(NT), shm, st, a);
            return hipGetLastError();
        }
    }
    if constexpr ((P == P64 || P == P32) && HOP) {
        if (a.blk) {   // FP64: the shared spinors, then one phase's links and a spare record
            const size_t links = P == P64 ? (size_t)(2 * a.NS + 1) * LinkLds<P, 0>::LB
                                          : stage_bytes(LinkLds<P, 0>::LB, a.NS);
            const size_t shm = std::max(tile, links + share_bytes(P, false, NT));
            hipLaunchKernelGGL((k_hop<P, DAG, HOP, 0, false, true>), dim3(nblk), dim3(NT), shm, st, a);
            return hipGetLastError();
        }
    }
    const size_t shm = HOP ? std::max(tile, stage_bytes(LinkLds<P, 0>::LB, a.NS)) : tile;
    hipLaunchKernelGGL((k_hop<P, DAG, HOP, 0>), dim3(nblk), dim3(NT), shm, st, a);
    return hipGetLastError();
}

// Hop with dense 5D blocks (kind-3 Op5s), for D_EOFA's even-odd form: FP64,
// FP32, or FP16 (matrix cores when the compact links are given)
template <int P, bool DAG, bool HOP>
static hipError_t launch_hop_dense_t(const HopArgs& a, int nblk, hipStream_t st) {
    using A = typename PT<P>::A;
    const int NT = a.NS * a.Ls;
    const size_t tile = (size_t)STR * NT * sizeof(A);
    if constexpr (P == P16 && HOP) {
        if (a.frag) {
            const size_t shm = std::max(tile, stage_bytes(LinkLds<P, 1>::LB, a.NS));
            if (a.depth >= 4) hipLaunchKernelGGL((k_hop<P, DAG, HOP, 4, true>), dim3(nblk), dim3(NT), shm, st, a);
            else if (a.depth == 3) hipLaunchKernelGGL((k_hop<P, DAG, HOP, 3, true>), dim3(nblk), dim3(NT), shm, st, a);
            else hipLaunchKernelGGL((k_hop<P, DAG, HOP, 2, true>), dim3(nblk), dim3(NT), shm, st, a);
            return hipGetLastError();
        }
    }
    const size_t shm = HOP ? std::max(tile, stage_bytes(LinkLds<P, 0>::LB, a.NS)) : tile;
    hipLaunchKernelGGL((k_hop<P, DAG, HOP, 0, true>), dim3(nblk), dim3(NT), shm, st, a);
    return hipGetLastError();
}

hipError_t launch_hop_dense(int prec, bool dag, bool hop, const HopArgs& a, int nblk, hipStream_t st) {
    if (!a.dmat) return hipErrorInvalidValue;
    if (prec == P64) {
        if (hop) return dag ? launch_hop_dense_t<P64, true, true>(a, nblk, st)
                            : launch_hop_dense_t<P64, false, true>(a, nblk, st);
        return launch_hop_dense_t<P64, false, false>(a, nblk, st);
    }
    if (prec == P32) {
        if (hop) return dag ? launch_hop_dense_t<P32, true, true>(a, nblk, st)
                            : launch_hop_dense_t<P32, false, true>(a, nblk, st);
        return launch_hop_dense_t<P32, false, false>(a, nblk, st);
    }
    if (prec == P16) {
        if (hop) return dag ? launch_hop_dense_t<P16, true, true>(a, nblk, st)
                            : launch_hop_dense_t<P16, false, true>(a, nblk, st);
        return launch_hop_dense_t<P16, false, false>(a, nblk, st);
    }
    return hipErrorInvalidValue;
}

// Workgroups per CU of the hop kernel (the K1 form: hop plus a column
// sweep) in its per-site or block-sharing form, as the runtime's occupancy
// calculator gives them for NS sites of Ls slices per workgroup; 0 on error.
// The block form needs more LDS, which lowers the occupancy where the links
// of many sites already fill it (small Ls).
template <int P, int MF, bool BLK>
static int hop_wg_per_cu(int NS, int Ls) {
    using A = typename PT<P>::A;
    const int NT = NS * Ls;
    const size_t tile = (size_t)STR * NT * sizeof(A);
    const size_t stage = (BLK && P == P64) ? (size_t)(2 * NS + 1) * LinkLds<P, 0>::LB
                                           : stage_bytes(LinkLds<P, MF ? 1 : 0>::LB, NS);
    const size_t shm = std::max(tile, stage + (BLK ? share_bytes(P, MF != 0, NT) : 0));
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_hop<P, false, true, MF, false, BLK>),
                                                     NT, shm) != hipSuccess)
        return 0;
    return n;
}

int hop_occupancy(int prec, bool mfma, bool blk, int NS, int Ls) {
    if (prec == P16 && mfma) return blk ? hop_wg_per_cu<P16, 3, true>(NS, Ls) : hop_wg_per_cu<P16, 3, false>(NS, Ls);
    if (prec == PB16 && mfma) return blk ? hop_wg_per_cu<PB16, 3, true>(NS, Ls) : hop_wg_per_cu<PB16, 3, false>(NS, Ls);
    if (prec == P32) return blk ? hop_wg_per_cu<P32, 0, true>(NS, Ls) : hop_wg_per_cu<P32, 0, false>(NS, Ls);
    if (prec == P64) return blk ? hop_wg_per_cu<P64, 0, true>(NS, Ls) : hop_wg_per_cu<P64, 0, false>(NS, Ls);
    return 0;
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

hipError_t launch_pupdate(int prec, const void* z, const float* zn, const void* po, const float* pon,
                          void* p, float* pn, void* pt,
                          float* ptn, const double* sc, int i_new, int i_old, int first, int Vh,
                          int Ls, int NS, size_t N, double b5, double c5, double mp, double mm,
                          int nblk, hipStream_t st) {
    const int NT = NS * Ls;
    switch (prec) {
#define EOFA_CASE(PP)                                                                         \
    case PP: {                                                                                \
        const size_t shm = (size_t)STR * NT * sizeof(typename PT<PP>::A);                     \
        hipLaunchKernelGGL((k_pupdate<PP>), dim3(nblk), dim3(NT), shm, st, z, zn, po, pon, p, pn, pt, \
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
