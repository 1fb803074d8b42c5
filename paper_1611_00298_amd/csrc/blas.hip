// blas.hip -- CG vector updates, FP64 reductions and precision conversion.
//
// Reductions are deterministic: every workgroup writes one FP64 partial
// (wavefront xor-shuffle tree, then a fixed-order sum over wavefronts) and
// a single-workgroup kernel sums the partials in a fixed order into a
// device scalar slot.  CG scalars (alpha, beta) are formed on the device
// from those slots, so no host round trip sits between the kernels.
#include "internal.h"

namespace eofa {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// workgroup sum of x (fixed order), written by thread 0 to *dst
__device__ __forceinline__ void block_store_sum(double x, double* dst) {
    __shared__ double red[16];
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += red[i];
        *dst = t;
    }
}

// out[slot] = sum of partial[0..n) (one workgroup of 1024).  Thread j sums
// partial[j], partial[j + 1024], ... in that order; the loads are issued 8 at
// a time so that one workgroup is not bound by the latency of a chain of
// dependent loads (a hop leaves one partial per workgroup: 55296 at 24^3x64).
__global__ void __launch_bounds__(1024) k_reduce(const double* __restrict__ partial, int n,
                                                 double* out, int slot) {
    // each work-item adds its elements in index order; 32 loads are in
    // flight at a time (a hop's 55 296 partials take two batches)
    double t = 0;
    const int step = blockDim.x;
    int i = threadIdx.x;
    for (; i + 31 * step < n; i += 32 * step) {
        double v[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) v[q] = partial[i + q * step];
#pragma unroll
        for (int q = 0; q < 32; ++q) t += v[q];
    }
    for (; i + 7 * step < n; i += 8 * step) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = partial[i + q * step];
#pragma unroll
        for (int q = 0; q < 8; ++q) t += v[q];
    }
    for (; i < n; i += step) t += partial[i];
    block_store_sum(t, out + slot);
}

// r -= alpha w ; partial |r|^2 ; alpha = sc[i_num] / sc[i_den], also kept in
// sc[i_save] for the batched solution update
template <int P>
__global__ void __launch_bounds__(256) k_r_update(void* r, float* rn, const void* w, const float* wn,
                                                  double* sc, int i_num, int i_den, int i_save,
                                                  size_t n5, size_t N, double* partial) {
    using A = typename PT<P>::A;
    const double alpha_d = sc[i_num] / sc[i_den];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[i_save] = alpha_d;
    const A alpha = (A)alpha_d;
    double acc = 0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        A wv[24], rv[24];
        ld_spinor<P>(w, wn, N, n, wv);
        ld_spinor<P>(r, rn, N, n, rv);
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            rv[k] = fmadd(-alpha, wv[k], rv[k]);
            acc += (double)rv[k] * (double)rv[k];
        }
        st_spinor<P>(r, rn, N, n, rv);
    }
    block_store_sum(acc, partial + blockIdx.x);
}

// x += sum_j alpha_j p_j over a batch of saved search directions
struct PBatch {
    const void* p[XBATCH];
    const float* pn[XBATCH];
    int slot[XBATCH];   // alpha_j = sc[slot[j]]
    int cnt;
};

template <int P, int PX>
__global__ void __launch_bounds__(256) k_x_batch(void* x, float* xn, const PBatch b, const double* sc,
                                                 size_t n5, size_t N) {
    using A = typename PT<P>::A;
    using AX = typename PT<PX>::A;
    AX al[XBATCH];
#pragma unroll
    for (int j = 0; j < XBATCH; ++j) al[j] = j < b.cnt ? (AX)sc[b.slot[j]] : AX(0);
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        AX xv[24];
        ld_spinor<PX>(x, xn, N, n, xv);
#pragma unroll
        for (int j = 0; j < XBATCH; ++j) {
            if (j < b.cnt) {
                A pv[24];
                ld_spinor<P>(b.p[j], b.pn[j], N, n, pv);
#pragma unroll
                for (int k = 0; k < 24; ++k) xv[k] = fmadd(al[j], (AX)pv[k], xv[k]);
            }
        }
        st_spinor<PX>(x, xn, N, n, xv);
    }
}

// partial |f|^2
template <int P>
__global__ void __launch_bounds__(256) k_norm2(const void* f, const float* fn, size_t n5, size_t N,
                                               double* partial) {
    using A = typename PT<P>::A;
    double acc = 0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        A v[24];
        ld_spinor<P>(f, fn, N, n, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc += (double)v[k] * (double)v[k];
    }
    block_store_sum(acc, partial + blockIdx.x);
}

// out = in, changing precision
template <int PI, int PO>
__global__ void __launch_bounds__(256) k_convert(const void* in, const float* inn, void* out,
                                                 float* outn, size_t n5, size_t N) {
    using AI = typename PT<PI>::A;
    using AO = typename PT<PO>::A;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        AI v[24];
        AO o[24];
        ld_spinor<PI>(in, inn, N, n, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] = (AO)v[k];
        st_spinor<PO>(out, outn, N, n, o);
    }
}

// xhi += xlo ; xlo = 0
template <int PX>
__global__ void __launch_bounds__(256) k_accum_hi(void* xhi, void* xlo, float* xlon, size_t n5,
                                                  size_t N) {
    using AX = typename PT<PX>::A;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        double h[24];
        AX l[24];
        ld_spinor<P64>(xhi, nullptr, N, n, h);
        ld_spinor<PX>(xlo, xlon, N, n, l);
#pragma unroll
        for (int k = 0; k < 24; ++k) { h[k] += (double)l[k]; l[k] = 0; }
        st_spinor<P64>(xhi, nullptr, N, n, h);
        st_spinor<PX>(xlo, xlon, N, n, l);
    }
}

template <int P>
__global__ void __launch_bounds__(256) k_zero(void* f, float* fn, size_t n5, size_t N) {
    using A = typename PT<P>::A;
    A v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x)
        st_spinor<P>(f, fn, N, n, v);
}

// partial Re <a, b> into partial[block] and Im <a, b> into partial[nblk + block]
// (FP64 half fields; <a, b> = sum conj(a) b)
__global__ void __launch_bounds__(256) k_cdot64(const void* a, const void* b, size_t n5, size_t N,
                                                double* partial) {
    double re = 0, im = 0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        double x[24], y[24];
        ld_spinor<P64>(a, nullptr, N, n, x);
        ld_spinor<P64>(b, nullptr, N, n, y);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            re += x[2 * k] * y[2 * k] + x[2 * k + 1] * y[2 * k + 1];
            im += x[2 * k] * y[2 * k + 1] - x[2 * k + 1] * y[2 * k];
        }
    }
    block_store_sum(re, partial + blockIdx.x);
    __syncthreads();   // block_store_sum's LDS is reused
    block_store_sum(im, partial + gridDim.x + blockIdx.x);
}

// x += (cr + i ci) y   (FP64 half fields)
__global__ void __launch_bounds__(256) k_caxpy64(void* x, const void* y, double cr, double ci, size_t n5,
                                                 size_t N) {
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        double u[24], v[24];
        ld_spinor<P64>(x, nullptr, N, n, u);
        ld_spinor<P64>(y, nullptr, N, n, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            u[2 * k] += cr * v[2 * k] - ci * v[2 * k + 1];
            u[2 * k + 1] += cr * v[2 * k + 1] + ci * v[2 * k];
        }
        st_spinor<P64>(x, nullptr, N, n, u);
    }
}

// CG step of the dense D_EOFA solve (FP64, or FP32 inside the mixed solve):
// x += alpha p ; s -= alpha w ; per-workgroup partials of |s|^2 in FP64
// (one pass instead of two axpys and a norm)
// x is held in PX (FP32 when p, s and w are 16-bit); FP16 fields carry their
// per-site norms
template <int P, int PX>
__global__ void __launch_bounds__(256) k_cg_step(void* x, const void* p, const float* pn, void* s, float* sn,
                                                 const void* w, const float* wn, double alpha_d, size_t n5,
                                                 size_t N, double* partial) {
    using A = typename PT<P>::A;
    using AX = typename PT<PX>::A;
    const A alpha = (A)alpha_d;
    double acc = 0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < n5;
         n += (size_t)gridDim.x * blockDim.x) {
        A u[24], v[24];
        AX xv[24];
        ld_spinor<PX>(x, nullptr, N, n, xv);
        ld_spinor<P>(p, pn, N, n, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) xv[k] = fmadd((AX)alpha, (AX)v[k], xv[k]);
        st_spinor<PX>(x, nullptr, N, n, xv);
        ld_spinor<P>(s, sn, N, n, u);
        ld_spinor<P>(w, wn, N, n, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            u[k] = fmadd(-alpha, v[k], u[k]);
            acc = fma((double)u[k], (double)u[k], acc);
        }
        st_spinor<P>(s, sn, N, n, u);
    }
    block_store_sum(acc, partial + blockIdx.x);
}

// ---------------------------------------------------------------------------
// launchers (grid: a fixed number of workgroups, grid-stride loops)
// ---------------------------------------------------------------------------
int blas_blocks(size_t n5) {
    size_t b = (n5 + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_cdot64(const void* a, const void* b, size_t n5, size_t N, double* partial, int nblk,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_cdot64, dim3(nblk), dim3(256), 0, st, a, b, n5, N, partial);
    return hipGetLastError();
}

hipError_t launch_caxpy64(void* x, const void* y, double cr, double ci, size_t n5, size_t N, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_caxpy64, dim3(nblk), dim3(256), 0, st, x, y, cr, ci, n5, N);
    return hipGetLastError();
}

hipError_t launch_cg_step(int prec, void* x, const void* p, const float* pn, void* s, float* sn, const void* w,
                          const float* wn, double alpha, size_t n5, size_t N, double* partial, int nblk,
                          hipStream_t st) {
    if (prec == P64)
        hipLaunchKernelGGL((k_cg_step<P64, P64>), dim3(nblk), dim3(256), 0, st, x, p, pn, s, sn, w, wn, alpha, n5,
                           N, partial);
    else if (prec == P32)
        hipLaunchKernelGGL((k_cg_step<P32, P32>), dim3(nblk), dim3(256), 0, st, x, p, pn, s, sn, w, wn, alpha, n5,
                           N, partial);
    else if (prec == P16)
        hipLaunchKernelGGL((k_cg_step<P16, P32>), dim3(nblk), dim3(256), 0, st, x, p, pn, s, sn, w, wn, alpha, n5,
                           N, partial);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int n, double* out, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, n, out, slot);
    return hipGetLastError();
}

hipError_t launch_r_update(int prec, void* r, float* rn, const void* w, const float* wn, double* sc,
                           int i_num, int i_den, int i_save, size_t n5, size_t N, double* partial,
                           int nblk, hipStream_t st) {
    switch (prec) {
    case P64: hipLaunchKernelGGL((k_r_update<P64>), dim3(nblk), dim3(256), 0, st, r, rn, w, wn, sc, i_num, i_den, i_save, n5, N, partial); break;
    case P32: hipLaunchKernelGGL((k_r_update<P32>), dim3(nblk), dim3(256), 0, st, r, rn, w, wn, sc, i_num, i_den, i_save, n5, N, partial); break;
    case P16: hipLaunchKernelGGL((k_r_update<P16>), dim3(nblk), dim3(256), 0, st, r, rn, w, wn, sc, i_num, i_den, i_save, n5, N, partial); break;
    case PB16: hipLaunchKernelGGL((k_r_update<PB16>), dim3(nblk), dim3(256), 0, st, r, rn, w, wn, sc, i_num, i_den, i_save, n5, N, partial); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_x_batch(int prec, void* x, float* xn, const void* const* p, const float* const* pn,
                          const int* slots, int cnt, const double* sc, size_t n5, size_t N, int nblk,
                          hipStream_t st) {
    if (cnt < 1 || cnt > XBATCH) return hipErrorInvalidValue;
    PBatch b;
    for (int j = 0; j < XBATCH; ++j) {
        b.p[j] = j < cnt ? p[j] : nullptr;
        b.pn[j] = j < cnt ? pn[j] : nullptr;
        b.slot[j] = j < cnt ? slots[j] : 0;
    }
    b.cnt = cnt;
    switch (prec) {
    case P64: hipLaunchKernelGGL((k_x_batch<P64, P64>), dim3(nblk), dim3(256), 0, st, x, xn, b, sc, n5, N); break;
    case P32: hipLaunchKernelGGL((k_x_batch<P32, P32>), dim3(nblk), dim3(256), 0, st, x, xn, b, sc, n5, N); break;
    case P16: hipLaunchKernelGGL((k_x_batch<P16, P32>), dim3(nblk), dim3(256), 0, st, x, xn, b, sc, n5, N); break;
    case PB16: hipLaunchKernelGGL((k_x_batch<PB16, P32>), dim3(nblk), dim3(256), 0, st, x, xn, b, sc, n5, N); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_norm2(int prec, const void* f, const float* fn, size_t n5, size_t N,
                        double* partial, int nblk, hipStream_t st) {
    switch (prec) {
    case P64: hipLaunchKernelGGL((k_norm2<P64>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N, partial); break;
    case P32: hipLaunchKernelGGL((k_norm2<P32>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N, partial); break;
    case P16: hipLaunchKernelGGL((k_norm2<P16>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N, partial); break;
    case PB16: hipLaunchKernelGGL((k_norm2<PB16>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N, partial); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PI>
static hipError_t convert_from(int po, const void* in, const float* inn, void* out, float* outn,
                               size_t n5, size_t N, int nblk, hipStream_t st) {
    switch (po) {
    case P64: hipLaunchKernelGGL((k_convert<PI, P64>), dim3(nblk), dim3(256), 0, st, in, inn, out, outn, n5, N); break;
    case P32: hipLaunchKernelGGL((k_convert<PI, P32>), dim3(nblk), dim3(256), 0, st, in, inn, out, outn, n5, N); break;
    case P16: hipLaunchKernelGGL((k_convert<PI, P16>), dim3(nblk), dim3(256), 0, st, in, inn, out, outn, n5, N); break;
    case PB16: hipLaunchKernelGGL((k_convert<PI, PB16>), dim3(nblk), dim3(256), 0, st, in, inn, out, outn, n5, N); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int pi, int po, const void* in, const float* inn, void* out, float* outn,
                          size_t n5, size_t N, int nblk, hipStream_t st) {
    switch (pi) {
    case P64: return convert_from<P64>(po, in, inn, out, outn, n5, N, nblk, st);
    case P32: return convert_from<P32>(po, in, inn, out, outn, n5, N, nblk, st);
    case P16: return convert_from<P16>(po, in, inn, out, outn, n5, N, nblk, st);
    case PB16: return convert_from<PB16>(po, in, inn, out, outn, n5, N, nblk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_accum_hi(int px, void* xhi, void* xlo, float* xlon, size_t n5, size_t N, int nblk,
                           hipStream_t st) {
    switch (px) {
    case P64: hipLaunchKernelGGL((k_accum_hi<P64>), dim3(nblk), dim3(256), 0, st, xhi, xlo, xlon, n5, N); break;
    case P32: hipLaunchKernelGGL((k_accum_hi<P32>), dim3(nblk), dim3(256), 0, st, xhi, xlo, xlon, n5, N); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero(int prec, void* f, float* fn, size_t n5, size_t N, int nblk, hipStream_t st) {
    switch (prec) {
    case P64: hipLaunchKernelGGL((k_zero<P64>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N); break;
    case P32: hipLaunchKernelGGL((k_zero<P32>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N); break;
    case P16: hipLaunchKernelGGL((k_zero<P16>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N); break;
    case PB16: hipLaunchKernelGGL((k_zero<PB16>), dim3(nblk), dim3(256), 0, st, f, fn, n5, N); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace eofa
