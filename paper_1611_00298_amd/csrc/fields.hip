// fields.hip -- ingest and layout conversion, the EOFA sources and action.
//
// Natural layouts (complex128): U[mu][i][3][3], phi[i][4][3], psi[s][i][4][3]
// with i = x + Lx*(y + Ly*(z + Lz*t)).  Device layouts: see internal.h.
#include "internal.h"

namespace eofa {

// Links of both output parities with -1/2 and the boundary sign folded in,
// and the neighbour table.  One work-item per (parity, cb).
__global__ void k_ingest_gauge(const double2* __restrict__ U, double2* __restrict__ G,
                               int* __restrict__ nbr, Geo g) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.Vh) return;
    const int p = t / g.Vh, cb = t - p * g.Vh;
    int c[4];
    const int i = natural_site(g, p, cb, c);
    double2* Gp = G + (size_t)p * 8 * 9 * g.Vh;
    int* np = nbr + (size_t)p * 8 * g.Vh;
    for (int d = 0; d < 8; ++d) {
        const int mu = d & 3;
        const bool fwd = d < 4;
        int e[4] = {c[0], c[1], c[2], c[3]};
        double sign = 1.0;
        e[mu] += fwd ? 1 : -1;
        if (e[mu] >= g.L[mu]) { e[mu] -= g.L[mu]; if (mu == 3 && g.aperiodic) sign = -1.0; }
        if (e[mu] < 0)        { e[mu] += g.L[mu]; if (mu == 3 && g.aperiodic) sign = -1.0; }
        const int j = index4(g, e);
        np[(size_t)d * g.Vh + cb] = j >> 1;
        const double f = -0.5 * sign;
        const double2* src = U + ((size_t)mu * g.V + (fwd ? i : j)) * 9;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double2 u;
                if (fwd) u = src[3 * a + b];
                else { double2 q = src[3 * b + a]; u = make_double2(q.x, -q.y); }
                Gp[((size_t)d * 9 + 3 * a + b) * g.Vh + cb] = make_double2(f * u.x, f * u.y);
            }
    }
}

// FP64 links -> lower-precision links (n complex numbers)
template <int PO>
__global__ void k_gauge_convert(const double2* __restrict__ in, void* __restrict__ out, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
        const double2 u = in[k];
        if constexpr (PO == P32) ((float2*)out)[k] = make_float2((float)u.x, (float)u.y);
        else if constexpr (PO == P16) ((uint32_t*)out)[k] = f2h((float)u.x) | (f2h((float)u.y) << 16);
        else ((uint32_t*)out)[k] = f2b((float)u.x) | (f2b((float)u.y) << 16);
    }
}

// FP64 links -> compact 16-bit links for the matrix-core hop, [p][d][Vh][9]
// complex numbers as (re, im) pairs of FP16 (bf = 0) or BF16 (bf = 1), 36
// bytes per link; the hop expands them into the rows of the real 6x6 form
// when it stages them in LDS.  One work-item per (p, d, cb).
__global__ void k_gauge_c16(const double2* __restrict__ in, uint32_t* __restrict__ out, int Vh, int bf) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * 8 * Vh) return;
    const int pd = t / Vh, cb = t - pd * Vh;
    uint32_t* o = out + ((size_t)pd * Vh + cb) * 9;
    for (int k = 0; k < 9; ++k) {
        const double2 u = in[((size_t)pd * 9 + k) * Vh + cb];
        o[k] = bf ? (f2b((float)u.x) | (f2b((float)u.y) << 16)) : (f2h((float)u.x) | (f2h((float)u.y) << 16));
    }
}

// natural 5D complex128 <-> FP64 device half fields (both parities)
__global__ void k_nat5_to_dev(const double2* __restrict__ nat, double2* __restrict__ de,
                              double2* __restrict__ dodd, Geo g, size_t N) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t nh = (size_t)g.Vh * g.Ls;
    if (t >= 2 * nh) return;
    const int p = (int)(t / nh);
    const size_t r = t - p * nh;
    const int cb = (int)(r / g.Ls), s = (int)(r - (size_t)cb * g.Ls);
    int c[4];
    const int i = natural_site(g, p, cb, c);
    const double2* src = nat + ((size_t)s * g.V + i) * 12;
    double2* dst = p ? dodd : de;
    for (int k = 0; k < 12; ++k) dst[k * N + r] = src[k];
}

__global__ void k_dev_to_nat5(double2* __restrict__ nat, const double2* __restrict__ de,
                              const double2* __restrict__ dodd, Geo g, size_t N) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t nh = (size_t)g.Vh * g.Ls;
    if (t >= 2 * nh) return;
    const int p = (int)(t / nh);
    const size_t r = t - p * nh;
    const int cb = (int)(r / g.Ls), s = (int)(r - (size_t)cb * g.Ls);
    int c[4];
    const int i = natural_site(g, p, cb, c);
    double2* dst = nat + ((size_t)s * g.V + i) * 12;
    const double2* src = p ? dodd : de;
    for (int k = 0; k < 12; ++k) dst[k] = src[k * N + r];
}

// Cayley-form sources of the two EOFA systems (footnote of Section 5.1):
//   b_L = g5 R5 Omega_- P_- phi : b_L(s) = -Omega_-(Ls-1-s) phi_lower
//   b_R = g5 R5 Omega_+ P_+ phi : b_R(s) = +Omega_-(s) phi_upper
// (Omega_+ = R5 Omega_-; gamma_5 = diag(1,1,-1,-1)).
__global__ void k_eofa_source(const double2* __restrict__ phi, const double* __restrict__ om,
                              double2* bLe, double2* bLo, double2* bRe, double2* bRo, Geo g,
                              size_t N) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t nh = (size_t)g.Vh * g.Ls;
    if (t >= 2 * nh) return;
    const int p = (int)(t / nh);
    const size_t r = t - p * nh;
    const int cb = (int)(r / g.Ls), s = (int)(r - (size_t)cb * g.Ls);
    int c[4];
    const int i = natural_site(g, p, cb, c);
    const double2* f = phi + (size_t)i * 12;
    const double wl = -om[g.Ls - 1 - s], wr = om[s];
    double2* bL = p ? bLo : bLe;
    double2* bR = p ? bRo : bRe;
    const double2 z = make_double2(0.0, 0.0);
    for (int k = 0; k < 6; ++k) {
        const double2 up = f[k], lo = f[6 + k];
        bL[k * N + r] = z;
        bL[(6 + k) * N + r] = make_double2(wl * lo.x, wl * lo.y);
        bR[k * N + r] = make_double2(wr * up.x, wr * up.y);
        bR[(6 + k) * N + r] = z;
    }
}

// Action of eq. (2.5): M_EOFA phi = phi - k P_- Omega_-^dag chi_L + k P_+ Omega_+^dag chi_R,
// S = phi^dag M_EOFA phi.  One work-item per natural 4D site; chi natural.
__global__ void __launch_bounds__(256) k_eofa_action(const double2* __restrict__ phi,
                                                     const double2* __restrict__ chiL,
                                                     const double2* __restrict__ chiR,
                                                     const double* __restrict__ om, double k,
                                                     double2* Mphi, double* partial, int V, int Ls) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0;
    if (i < V) {
        double2 aL[6], aR[6];
        for (int q = 0; q < 6; ++q) { aL[q] = make_double2(0, 0); aR[q] = make_double2(0, 0); }
        for (int s = 0; s < Ls; ++s) {
            const double wL = om[s], wR = om[Ls - 1 - s];   // Omega_-(s), Omega_+(s)
            const double2* cl = chiL + ((size_t)s * V + i) * 12;
            const double2* cr = chiR + ((size_t)s * V + i) * 12;
            for (int q = 0; q < 6; ++q) {
                const double2 l = cl[6 + q], rr = cr[q];
                aL[q].x += wL * l.x; aL[q].y += wL * l.y;
                aR[q].x += wR * rr.x; aR[q].y += wR * rr.y;
            }
        }
        const double2* f = phi + (size_t)i * 12;
        for (int q = 0; q < 12; ++q) {
            const double2 fv = f[q];
            double2 m;
            if (q < 6) m = make_double2(fv.x + k * aR[q].x, fv.y + k * aR[q].y);
            else m = make_double2(fv.x - k * aL[q - 6].x, fv.y - k * aL[q - 6].y);
            acc += fv.x * m.x + fv.y * m.y;   // Re(conj(phi) M phi)
            if (Mphi) Mphi[(size_t)i * 12 + q] = m;
        }
    }
    __shared__ double red[8];
    double x = acc;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_ingest_gauge(const void* U, void* G, int* nbr, const int L[4], int Ls, int aperiodic,
                               hipStream_t st) {
    Geo g{{L[0], L[1], L[2], L[3]}, L[0] * L[1] * L[2] * L[3], L[0] * L[1] * L[2] * L[3] / 2, Ls, aperiodic};
    const int n = 2 * g.Vh;
    hipLaunchKernelGGL(k_ingest_gauge, dim3((n + 255) / 256), dim3(256), 0, st, (const double2*)U,
                       (double2*)G, nbr, g);
    return hipGetLastError();
}

hipError_t launch_gauge_convert(int po, const void* in, void* out, size_t n, hipStream_t st) {
    const int nblk = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    switch (po) {
    case P32: hipLaunchKernelGGL((k_gauge_convert<P32>), dim3(nblk), dim3(256), 0, st, (const double2*)in, out, n); break;
    case P16: hipLaunchKernelGGL((k_gauge_convert<P16>), dim3(nblk), dim3(256), 0, st, (const double2*)in, out, n); break;
    case PB16: hipLaunchKernelGGL((k_gauge_convert<PB16>), dim3(nblk), dim3(256), 0, st, (const double2*)in, out, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static Geo make_geo(const int L[4], int Ls) {
    const int V = L[0] * L[1] * L[2] * L[3];
    return Geo{{L[0], L[1], L[2], L[3]}, V, V / 2, Ls, 0};
}

hipError_t launch_nat5_to_dev(const void* nat, void* de, void* dodd, const int L[4], int Ls, size_t N,
                              hipStream_t st) {
    Geo g = make_geo(L, Ls);
    const size_t n = 2 * (size_t)g.Vh * Ls;
    hipLaunchKernelGGL(k_nat5_to_dev, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const double2*)nat, (double2*)de, (double2*)dodd, g, N);
    return hipGetLastError();
}

hipError_t launch_dev_to_nat5(void* nat, const void* de, const void* dodd, const int L[4], int Ls,
                              size_t N, hipStream_t st) {
    Geo g = make_geo(L, Ls);
    const size_t n = 2 * (size_t)g.Vh * Ls;
    hipLaunchKernelGGL(k_dev_to_nat5, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (double2*)nat, (const double2*)de, (const double2*)dodd, g, N);
    return hipGetLastError();
}

hipError_t launch_eofa_source(const void* phi, const double* om, void* bLe, void* bLo, void* bRe,
                              void* bRo, const int L[4], int Ls, size_t N, hipStream_t st) {
    Geo g = make_geo(L, Ls);
    const size_t n = 2 * (size_t)g.Vh * Ls;
    hipLaunchKernelGGL(k_eofa_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const double2*)phi, om, (double2*)bLe, (double2*)bLo, (double2*)bRe,
                       (double2*)bRo, g, N);
    return hipGetLastError();
}

// Heatbath of eq. (3.1).  phi = c0 eta over the 4D field (n complex numbers).
__global__ void k_hb_init(const double2* __restrict__ eta, double2* __restrict__ phi, double c0,
                          size_t n) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double2 e = eta[t];
    phi[t] = make_double2(c0 * e.x, c0 * e.y);
}

// phi(x) += coef P Omega^dag chi(x) = coef sum_s Omega(s) P chi(x, s), with chi
// a solution in the device layout (parity halves ce/co, component-major).
// lower: P_- (spins 2, 3) with Omega_-(s) = om[s]; else P_+ (spins 0, 1)
// with Omega_+(s) = om[Ls - 1 - s].  One work-item per 4D site.
__global__ void k_hb_accum(double2* __restrict__ phi, const double2* __restrict__ ce,
                           const double2* __restrict__ co, const double* __restrict__ om,
                           double coef, int lower, Geo g, size_t N) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= 2 * (size_t)g.Vh) return;
    const int p = (int)(t / g.Vh);
    const int cb = (int)(t - (size_t)p * g.Vh);
    int c[4];
    const int i = natural_site(g, p, cb, c);
    const double2* src = p ? co : ce;
    const int k0 = lower ? 6 : 0;
    double2 acc[6];
    for (int q = 0; q < 6; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int s = 0; s < g.Ls; ++s) {
        const double w = lower ? om[s] : om[g.Ls - 1 - s];
        const size_t r = (size_t)cb * g.Ls + s;
        for (int q = 0; q < 6; ++q) {
            const double2 v = src[(size_t)(k0 + q) * N + r];
            acc[q].x += w * v.x;
            acc[q].y += w * v.y;
        }
    }
    double2* f = phi + (size_t)i * 12 + k0;
    for (int q = 0; q < 6; ++q) {
        const double2 o = f[q];
        f[q] = make_double2(o.x + coef * acc[q].x, o.y + coef * acc[q].y);
    }
}

// Lanczos on M_EOFA (4D fields, 12 complex per site).
// partial[block] = sum over the block's sites of Re <a, b>.
__global__ void __launch_bounds__(256) k_dot4(const double2* __restrict__ a,
                                              const double2* __restrict__ b, double* partial, int V) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0;
    if (i < V) {
        for (int q = 0; q < 12; ++q) {
            const double2 x = a[(size_t)i * 12 + q], y = b[(size_t)i * 12 + q];
            acc += x.x * y.x + x.y * y.y;
        }
    }
    __shared__ double red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// w = w - alpha v - beta vp (the three-term recurrence; vp may be NULL when beta = 0)
__global__ void k_lanczos_axpy(double2* __restrict__ w, const double2* __restrict__ v,
                               const double2* __restrict__ vp, double alpha, double beta, size_t n) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    double2 x = w[t];
    const double2 a = v[t];
    x.x -= alpha * a.x;
    x.y -= alpha * a.y;
    if (vp) {
        const double2 c = vp[t];
        x.x -= beta * c.x;
        x.y -= beta * c.y;
    }
    w[t] = x;
}

int dot4_blocks(int V) { return (V + 255) / 256; }

hipError_t launch_dot4(const void* a, const void* b, double* partial, int V, hipStream_t st) {
    hipLaunchKernelGGL(k_dot4, dim3(dot4_blocks(V)), dim3(256), 0, st, (const double2*)a,
                       (const double2*)b, partial, V);
    return hipGetLastError();
}

hipError_t launch_lanczos_axpy(void* w, const void* v, const void* vp, double alpha, double beta,
                               size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_lanczos_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (double2*)w, (const double2*)v, (const double2*)vp, alpha, beta, n);
    return hipGetLastError();
}

hipError_t launch_hb_init(const void* eta, void* phi, double c0, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_hb_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const double2*)eta, (double2*)phi, c0, n);
    return hipGetLastError();
}

hipError_t launch_hb_accum(void* phi, const void* ce, const void* co, const double* om, double coef,
                           int lower, const int L[4], int Ls, size_t N, hipStream_t st) {
    Geo g = make_geo(L, Ls);
    const size_t n = 2 * (size_t)g.Vh;
    hipLaunchKernelGGL(k_hb_accum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (double2*)phi, (const double2*)ce, (const double2*)co, om, coef, lower, g, N);
    return hipGetLastError();
}

// Links of a block traversal table in block-major order, for the
// block-sharing hops: record (p, b, d, j) = the link of direction d of the
// site in slot j of block b (sites[8 b + j]) for output parity p, the 8
// direction records of a block's 8 slots contiguous.  16-bit compact links
// (wide = 0): source [p][d][Vh][9] words, 36 B records; FP32 links (wide =
// 1): source [p][d][9][Vh] complex, 72 B records; FP64 links (wide = 2):
// the same source layout with 144 B records, in the phase order of the FP64
// block hop.  Padding slots get zeros.  One work-item per record.
__global__ void k_links_blocked(const void* __restrict__ src, void* __restrict__ dst,
                                const int* __restrict__ sites, int Vh, int nblk, int wide) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * nblk * 64) return;
    const int j = t & 7, d = (t >> 3) & 7, pb = t >> 6;
    const int p = pb / nblk, b = pb - p * nblk;
    const int site = sites[8 * b + j];
    if (wide == 2) {
        // FP64: records in phase order, (ph, k, j) with the direction of phase
        // ph, slot k for slot j's offsets (the FP64 block hop stages one
        // phase's 16 records at a time): phases 0, 1 the inside directions of
        // mu = 2 (ph mod 2) + k, phases 2, 3 the outside ones
        const int ph = (t >> 4) & 3, k2 = (t >> 3) & 1;
        const int off = (j << 1) | ((__popc(j) + p) & 1);
        const int mu = 2 * (ph & 1) + k2;
        const int din = mu + 4 * ((off >> mu) & 1);
        const int dd = ph < 2 ? din : din ^ 4;
        const double2* in = reinterpret_cast<const double2*>(src) + ((size_t)p * 8 + dd) * 9 * Vh;
        double2* out = reinterpret_cast<double2*>(dst) + (size_t)t * 9;
        for (int k = 0; k < 9; ++k) out[k] = site < Vh ? in[(size_t)k * Vh + site] : make_double2(0.0, 0.0);
    } else if (wide) {
        const float2* in = reinterpret_cast<const float2*>(src) + ((size_t)p * 8 + d) * 9 * Vh;
        float2* out = reinterpret_cast<float2*>(dst) + (size_t)t * 9;
        for (int k = 0; k < 9; ++k) out[k] = site < Vh ? in[(size_t)k * Vh + site] : make_float2(0.f, 0.f);
    } else {
        const uint32_t* in = reinterpret_cast<const uint32_t*>(src) + (((size_t)p * 8 + d) * Vh + site) * 9;
        uint32_t* out = reinterpret_cast<uint32_t*>(dst) + (size_t)t * 9;
        for (int k = 0; k < 9; ++k) out[k] = site < Vh ? in[k] : 0u;
    }
}

hipError_t launch_links_blocked(const void* src, void* dst, const int* sites, int Vh, int nslot, int wide,
                                hipStream_t st) {
    const int nblk = nslot / 8, n = 2 * nblk * 64;
    hipLaunchKernelGGL(k_links_blocked, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, sites, Vh, nblk, wide);
    return hipGetLastError();
}

hipError_t launch_gauge_c16(const void* in, void* out, int Vh, int bf, hipStream_t st) {
    const int n = 2 * 8 * Vh;
    hipLaunchKernelGGL(k_gauge_c16, dim3((n + 255) / 256), dim3(256), 0, st, (const double2*)in, (uint32_t*)out, Vh,
                       bf);
    return hipGetLastError();
}

int action_blocks(int V) { return (V + 255) / 256; }

hipError_t launch_eofa_action(const void* phi, const void* chiL, const void* chiR, const double* om,
                              double k, void* Mphi, double* partial, int V, int Ls, hipStream_t st) {
    hipLaunchKernelGGL(k_eofa_action, dim3(action_blocks(V)), dim3(256), 0, st, (const double2*)phi,
                       (const double2*)chiL, (const double2*)chiR, om, k, (double2*)Mphi, partial, V,
                       Ls);
    return hipGetLastError();
}

}  // namespace eofa
