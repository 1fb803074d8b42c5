// internal.h -- shared declarations of the gfx950 EOFA library (GPU side only).
//
// Device layout of a 5D fermion field: one checkerboard ("half field") of
// Vh = V/2 4D sites times Ls slices.  The 5D site index is n = cb*Ls + s
// with cb = i/2 the checkerboard index of natural site i, so the Ls slices
// of one 4D site are adjacent and a workgroup owns whole 4D sites.
// Components are stored as 16-byte blocks, block-major ("SoA of 16 B"):
//   FP64 : 12 blocks of double2 (one complex each)
//   FP32 :  6 blocks of float4  (two complex each)
//   FP16 :  3 blocks of 8 halves (four complex each) + one float norm per site
//   BF16 :  3 blocks of 8 bfloat16
// Block b of site n lives at base[b*N + n], N = padded number of 5D sites,
// so the lanes of a wavefront read consecutive 16-byte words.
//
// Gauge links for output parity p are stored per output site, already
// multiplied by -1/2 and by the boundary sign:
//   d = 0..3 : -1/2 sigma U_mu(x)          (hop from x+mu)
//   d = 4..7 : -1/2 sigma U_mu(x-mu)^dag   (hop from x-mu)
// as [p][d][9][Vh] complex numbers of the field precision.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace eofa {

enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };

template <int P> struct PT;
template <> struct PT<P64>  { using A = double; static constexpr int NB = 12; static constexpr int CB = 16; };
template <> struct PT<P32>  { using A = float;  static constexpr int NB = 6;  static constexpr int CB = 8; };
template <> struct PT<P16>  { using A = float;  static constexpr int NB = 3;  static constexpr int CB = 4; };
template <> struct PT<PB16> { using A = float;  static constexpr int NB = 3;  static constexpr int CB = 4; };

inline int nblocks_of(int p) { return p == P64 ? 12 : p == P32 ? 6 : 3; }
inline int complex_bytes(int p) { return p == P64 ? 16 : p == P32 ? 8 : 4; }
// algorithmic bytes of one 5D spinor site
inline int spinor_bytes(int p) { return p == P64 ? 192 : p == P32 ? 96 : p == P16 ? 52 : 48; }

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// 16-bit conversions
// ---------------------------------------------------------------------------
__device__ __forceinline__ float h2f(uint32_t bits16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}
__device__ __forceinline__ uint32_t f2h(float f) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
}
__device__ __forceinline__ float b2f(uint32_t bits16) {
    return __uint_as_float(bits16 << 16);
}
__device__ __forceinline__ uint32_t f2b(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// ---------------------------------------------------------------------------
// spinor load / store (24 reals: complex c = spin*3 + colour, re = 2c)
// ---------------------------------------------------------------------------
// Field accesses use a uniform (scalar) base per 16-byte block plus a
// 32-bit byte offset per lane, so the loads can use SGPR-base addressing.
template <typename T>
__device__ __forceinline__ const T& at(const void* base, size_t blk_bytes, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + blk_bytes + off);
}
template <typename T>
__device__ __forceinline__ T& at_mut(void* base, size_t blk_bytes, uint32_t off) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + blk_bytes + off);
}

// 16-byte block access; NT = non-temporal (streaming) hint for data that is
// touched once, so that it does not displace reused neighbour data in L2
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 ld16(const void* base, size_t blk, uint32_t off) {
    const u32x4_t* q = reinterpret_cast<const u32x4_t*>(reinterpret_cast<const char*>(base) + blk + off);
    u32x4_t v = NT ? __builtin_nontemporal_load(q) : *q;
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <bool NT>
__device__ __forceinline__ void st16(void* base, size_t blk, uint32_t off, uint4 t) {
    u32x4_t* q = reinterpret_cast<u32x4_t*>(reinterpret_cast<char*>(base) + blk + off);
    u32x4_t v = {t.x, t.y, t.z, t.w};
    if (NT) __builtin_nontemporal_store(v, q); else *q = v;
}
template <int P, bool NT = false>
__device__ __forceinline__ void ld_spinor(const void* __restrict__ base, const float* __restrict__ nrm,
                                          size_t N, size_t n, typename PT<P>::A (&v)[24]) {
    const uint32_t off = (uint32_t)n * 16u;
    const size_t bb = N * 16;
    if constexpr (P == P64) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 t = __builtin_bit_cast(double2, ld16<NT>(base, c * bb, off));
            v[2 * c] = t.x; v[2 * c + 1] = t.y;
        }
    } else if constexpr (P == P32) {
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            const float4 t = __builtin_bit_cast(float4, ld16<NT>(base, b * bb, off));
            v[4 * b] = t.x; v[4 * b + 1] = t.y; v[4 * b + 2] = t.z; v[4 * b + 3] = t.w;
        }
    } else {
        float sc = 1.0f;
        if constexpr (P == P16) sc = NT ? __builtin_nontemporal_load(nrm + n) : nrm[n];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const uint4 t = ld16<NT>(base, b * bb, off);
            uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (P == P16) {
                    v[8 * b + 2 * q] = h2f(w[q] & 0xffffu) * sc;
                    v[8 * b + 2 * q + 1] = h2f(w[q] >> 16) * sc;
                } else {
                    v[8 * b + 2 * q] = b2f(w[q] & 0xffffu);
                    v[8 * b + 2 * q + 1] = b2f(w[q] >> 16);
                }
            }
        }
    }
}

template <int P, bool NT = false>
__device__ __forceinline__ void st_spinor(void* __restrict__ base, float* __restrict__ nrm,
                                          size_t N, size_t n, const typename PT<P>::A (&v)[24]) {
    const uint32_t off = (uint32_t)n * 16u;
    const size_t bb = N * 16;
    if constexpr (P == P64) {
#pragma unroll
        for (int c = 0; c < 12; ++c)
            st16<NT>(base, c * bb, off, __builtin_bit_cast(uint4, make_double2(v[2 * c], v[2 * c + 1])));
    } else if constexpr (P == P32) {
#pragma unroll
        for (int b = 0; b < 6; ++b)
            st16<NT>(base, b * bb, off,
                     __builtin_bit_cast(uint4, make_float4(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3])));
    } else {
        float sc = 1.0f;
        if constexpr (P == P16) {
            float m = 0.0f;
#pragma unroll
            for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf(v[k]));
            if (NT) __builtin_nontemporal_store(m, nrm + n); else nrm[n] = m;
            sc = m > 0.0f ? 1.0f / m : 0.0f;
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (P == P16)
                    w[q] = f2h(v[8 * b + 2 * q] * sc) | (f2h(v[8 * b + 2 * q + 1] * sc) << 16);
                else
                    w[q] = f2b(v[8 * b + 2 * q]) | (f2b(v[8 * b + 2 * q + 1]) << 16);
            }
            st16<NT>(base, b * bb, off, make_uint4(w[0], w[1], w[2], w[3]));
        }
    }
}

// Raw 16-bit spinor load: the stored values without the FP16 site norm
// (returned separately, 1 for BF16), so that the norm can be applied after
// the spin projection on 12 instead of 24 numbers.
template <int P>
__device__ __forceinline__ float ld_spinor_raw(const void* __restrict__ base, const float* __restrict__ nrm,
                                               size_t N, size_t n, float (&v)[24]) {
    static_assert(P == P16 || P == PB16, "16-bit storage only");
    const uint32_t off = (uint32_t)n * 16u;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const uint4 t = at<uint4>(base, b * N * 16, off);
        uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (P == P16) {
                v[8 * b + 2 * q] = h2f(w[q] & 0xffffu);
                v[8 * b + 2 * q + 1] = h2f(w[q] >> 16);
            } else {
                v[8 * b + 2 * q] = b2f(w[q] & 0xffffu);
                v[8 * b + 2 * q + 1] = b2f(w[q] >> 16);
            }
        }
    }
    if constexpr (P == P16) return nrm[n];
    return 1.0f;
}

// ---------------------------------------------------------------------------
// links, [p][d][9][Vh] complex (row-major 3x3): FP64 fields use FP64 links;
// the FP32 and vector 16-bit paths use FP32 links (their bytes are shared by
// the Ls slices of a 4D site, so FP32 costs little traffic and saves the
// 16-bit conversions); the matrix-core paths use compact 16-bit copies.
// ---------------------------------------------------------------------------
constexpr int link_prec(int p) { return p == P64 ? P64 : P32; }

// Size of the static scratch array of the allocation-free MD update, in
// doubles: one partial sum per 256 links, so lattices of up to 2^20 4D
// sites (128 KiB per GPU).
constexpr int MD_SCRATCH_DOUBLES = 16384;
// search directions per batched solution update (x += sum_j alpha_j p_j)
constexpr int XBATCH = 16;

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that XCD x works on one contiguous range of
// logical blocks (neighbouring 4D sites then share an L2).
__device__ __forceinline__ int xcd_block(int nblk) {
    constexpr int NX = 8;
    const int b = blockIdx.x;
    const int per = nblk / NX, rem = nblk % NX;
    const int x = b % NX, q = b / NX;
    return x * per + (x < rem ? x : rem) + q;
}

// ---------------------------------------------------------------------------
// lattice geometry: natural index i = x + Lx*(y + Ly*(z + Lz*t)),
// checkerboard index cb = i/2 within parity p = (x+y+z+t) mod 2
// ---------------------------------------------------------------------------
struct Geo {
    int L[4];
    int V, Vh, Ls;
    int aperiodic;
};

// natural site index of checkerboard index cb with parity p
__device__ __forceinline__ int natural_site(const Geo& g, int p, int cb, int c[4]) {
    const int i0 = 2 * cb;
    int x0 = i0 % g.L[0];
    int rem = i0 / g.L[0];
    c[1] = rem % g.L[1];
    rem /= g.L[1];
    c[2] = rem % g.L[2];
    c[3] = rem / g.L[2];
    c[0] = x0 + ((p + c[1] + c[2] + c[3]) & 1);
    return i0 + (c[0] - x0);
}

__device__ __forceinline__ int index4(const Geo& g, const int c[4]) {
    return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------

// A 5D-local operator on the fifth dimension, per chirality:
//   kind 0: identity, 1: a + b S, 2: (a + b S)^-1,
// S = L (tr = 0) or L^T (tr = 1) with masses (m+, m-) of the launch.
struct Op5 {
    int kind;
    int tr;
    double a, b;
};

// out = C( ch * A(Dh in) + ca * B2(B(aux)) + cr * aux2 ), and optionally the
// per-workgroup partial sums of |out|^2.  A, C and B2 act through LDS column
// sweeps; B alone (B2 = 1) is a bidiagonal or identity op by row exchange.
struct HopArgs {
    const void* in; const float* in_nrm;
    void* out; float* out_nrm;
    const void* aux; const float* aux_nrm;
    const void* aux2; const float* aux2_nrm;
    const void* gauge;   // links of the output parity, [8][9][Vh]
    const int* nbr;      // neighbour cb index of the output parity, [8][Vh]
    const int* sites;    // traversal: slot lb*NS + sl -> output site, >= Vh for padding (nullable)
    const void* frag;    // compact FP16 links for the matrix-core path, [8][Vh][9] (re, im) halves (nullable)
    int depth;           // directions of operands kept in flight (matrix-core path)
    int par;             // parity of the output sites
    int blk;             // the site table lists whole 2x2x2x2 blocks, 8 slots each (block-sharing hops)
    const int* nbrb;     // with blk: neighbours of the table's blocks, [block][k][slot] (k = 0: x inside, 1-4: outside)
    const void* lnkb;    // with blk: the links in block-major order, [block][d][slot] records (FP32 or compact 16-bit)
    int Vh, Ls, NS;
    size_t N;
    double mp, mm;
    Op5 opA, opB, opC;
    Op5 opB2;            // if non-trivial, aux goes through a column sweep: ca B2(B(aux))
    double ch, ca, cr;
    double* partial;
    // optional device scalar: ch and ca are multiplied by alpha =
    // dsc[s_num] / dsc[s_den], which is also stored to dsc[s_alpha] (>= 0)
    double* dsc;
    int s_num, s_den, s_alpha;
    // dense 5D blocks of D_EOFA's even-odd form (the dense comparison path, FP64, FP32 or FP16):
    // [D5+, D5-, D5inv+, D5inv-], each Ls x Ls row major; an Op5 of kind 3
    // applies D5 (a = 0) or D5^-1 (a = 1), transposed when tr != 0
    const double* dmat;
};

}  // namespace eofa
