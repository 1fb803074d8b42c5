// api.cpp -- C ABI, context and workspaces, and the EOFA solver drivers.
//
// The solver follows Section 5.1 of the paper: the EOFA systems (eq. (5.1)
// with alpha_l in {0, -1}) are right-preconditioned into the Cayley form
// (H^-1 v = Dtilde D_DWF^-1 gamma_5 R_5 v), even-odd preconditioned, and
// solved by CGNR on the odd-site Schur complement
//   Mhat = M_ee - Dh_oe Dtilde M_ee^-1 Dh_eo Dtilde
// either in FP64 or with a reliable-update mixed-precision inner loop
// (FP32, FP16+norm or BF16 storage; FP64 reductions, FP64 solution and FP64
// residual recomputation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "eofa.h"
#include "internal.h"

namespace eofa {
hipError_t launch_hop(int prec, bool dag, bool hop, const HopArgs& a, int nblk, hipStream_t st);
int hop_occupancy(int prec, bool mfma, bool blk, int NS, int Ls);
hipError_t launch_pupdate(int prec, const void* z, const float* zn, const void* po, const float* pon,
                          void* p, float* pn, void* pt,
                          float* ptn, const double* sc, int i_new, int i_old, int first, int Vh,
                          int Ls, int NS, size_t N, double b5, double c5, double mp, double mm,
                          int nblk, hipStream_t st);
hipError_t launch_r_update(int prec, void* r, float* rn, const void* w, const float* wn, double* sc,
                           int i_num, int i_den, int i_save, size_t n5, size_t N, double* partial,
                           int nblk, hipStream_t st);
hipError_t launch_x_batch(int prec, void* x, float* xn, const void* const* p, const float* const* pn,
                          const int* slots, int cnt, const double* sc, size_t n5, size_t N, int nblk,
                          hipStream_t st);
int blas_blocks(size_t n5);
hipError_t launch_reduce(const double* partial, int n, double* out, int slot, hipStream_t st);
hipError_t launch_norm2(int prec, const void* f, const float* fn, size_t n5, size_t N,
                        double* partial, int nblk, hipStream_t st);
hipError_t launch_convert(int pi, int po, const void* in, const float* inn, void* out, float* outn,
                          size_t n5, size_t N, int nblk, hipStream_t st);
hipError_t launch_accum_hi(int px, void* xhi, void* xlo, float* xlon, size_t n5, size_t N, int nblk,
                           hipStream_t st);
hipError_t launch_zero(int prec, void* f, float* fn, size_t n5, size_t N, int nblk, hipStream_t st);
hipError_t launch_ingest_gauge(const void* U, void* G, int* nbr, const int L[4], int Ls, int aperiodic,
                               hipStream_t st);
hipError_t launch_gauge_convert(int po, const void* in, void* out, size_t n, hipStream_t st);
hipError_t launch_gauge_c16(const void* in, void* out, int Vh, int bf, hipStream_t st);
hipError_t launch_links_blocked(const void* src, void* dst, const int* sites, int Vh, int nslot, int wide,
                                hipStream_t st);
hipError_t launch_nat5_to_dev(const void* nat, void* de, void* dodd, const int L[4], int Ls, size_t N,
                              hipStream_t st);
hipError_t launch_dev_to_nat5(void* nat, const void* de, const void* dodd, const int L[4], int Ls,
                              size_t N, hipStream_t st);
hipError_t launch_eofa_source(const void* phi, const double* om, void* bLe, void* bLo, void* bRe,
                              void* bRo, const int L[4], int Ls, size_t N, hipStream_t st);
hipError_t launch_hb_init(const void* eta, void* phi, double c0, size_t n, hipStream_t st);
hipError_t launch_hb_accum(void* phi, const void* ce, const void* co, const double* om, double coef,
                           int lower, const int L[4], int Ls, size_t N, hipStream_t st);
void zolotarev_inv_sqrt(double lo, double hi, int n, double* alpha0, double* alpha, double* beta,
                        double* delta_out);
int dot4_blocks(int V);
hipError_t launch_cdot64(const void* a, const void* b, size_t n5, size_t N, double* partial, int nblk,
                         hipStream_t st);
hipError_t launch_caxpy64(void* x, const void* y, double cr, double ci, size_t n5, size_t N, int nblk,
                          hipStream_t st);
hipError_t launch_dot4(const void* a, const void* b, double* partial, int V, hipStream_t st);
hipError_t launch_lanczos_axpy(void* w, const void* v, const void* vp, double alpha, double beta,
                               size_t n, hipStream_t st);
int action_blocks(int V);
hipError_t launch_eofa_action(const void* phi, const void* chiL, const void* chiR, const double* om,
                              double k, void* Mphi, double* partial, int V, int Ls, hipStream_t st);
hipError_t launch_force(const void* U, const void* chiLe, const void* chiLo, const void* chiRe,
                        const void* chiRo, const int* nbr, const int* sites, double k, void* F, void* G,
                        const int L[4], int Ls, int aperiodic, int NS, int nblk, size_t N, hipStream_t st);
int md_blocks(int nlink);
hipError_t md_scratch_address(double** out);
hipError_t launch_md_update(void* U, void* P, const void* F, double dt_p, double dt_u, int nlink,
                            double* partial, hipStream_t st);
hipError_t launch_hop_dense(int prec, bool dag, bool hop, const HopArgs& a, int nblk, hipStream_t st);
hipError_t launch_cg_step(int prec, void* x, const void* p, const float* pn, void* s, float* sn, const void* w,
                          const float* wn, double alpha, size_t n5, size_t N, double* partial, int nblk,
                          hipStream_t st);
int gauge_action_blocks(int V);
hipError_t launch_gauge_force(const void* U, void* F, const int L[4], double beta, double c1, int accumulate,
                              hipStream_t st);
hipError_t launch_gauge_action(const void* U, const int L[4], double c1, double* partial, hipStream_t st);
}  // namespace eofa

using namespace eofa;

namespace {

thread_local std::string g_err;

struct Fail {
    int code;
};

[[noreturn]] void fail(int code, const std::string& msg) {
    g_err = msg;
    throw Fail{code};
}

void hipchk(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(EOFA_ENOMEM, std::string(what) + ": out of device memory");
        fail(EOFA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

// one checkerboard half of a 5D field in device layout
struct Half {
    void* d = nullptr;
    float* nrm = nullptr;
    int prec = -1;
};

enum Cls { C_HOP64 = 0, C_HOP32, C_HOP16, C_HOPB16, C_BLAS, C_FORCE, C_MD, C_GFORCE, C_GACTION, C_HOPDENSE,
           C_NCLS };
const char* cls_name[C_NCLS] = {"hop64", "hop32", "hop16", "hopb16", "blas", "force", "md",
                                "gauge_force", "gauge_action", "hop_dense"};

struct TimingRec {
    int cls;
    int ev;
    double bytes;
};

// Device address of the MD update's static scratch array, per GPU, taken
// once per device at context creation with that device current.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

void init_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) fail(EOFA_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return;
    double* p = nullptr;
    hipchk(md_scratch_address(&p), "hipGetSymbolAddress(scratch)");
    if (!p) fail(EOFA_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = p;
}

double* scratch_of(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < MAX_DEVICES ? g_scratch[dev] : nullptr;
}

}  // namespace

struct eofa_ctx {
    int dev = 0;
    hipStream_t st = nullptr;
    int L[4] = {0, 0, 0, 0};
    int Ls = 0, V = 0, Vh = 0, aperiodic = 1;
    double M5 = 0, alpha = 0, b5 = 0, c5 = 0, beta0 = 0, beta1 = 0;
    size_t n5 = 0, N = 0;
    int NS = 0, nblk_hop = 0, nblk_blas = 0;
    int* nbr = nullptr;
    int* sites[4] = {nullptr, nullptr, nullptr, nullptr};   // hop traversal (site per slot) per precision
    int blk[4] = {0, 0, 0, 0};   // the table lists whole 2x2x2x2 blocks (FP32 and matrix-core paths)
    int* nbrb[4] = {nullptr, nullptr, nullptr, nullptr};   // block-major neighbours of a block table
    int* fsites = nullptr;   // the per-site FP64 traversal (force kernel, dense hops)
    void* lnkb[4] = {nullptr, nullptr, nullptr, nullptr};  // block-major links of a block table (P32, P16, PB16)
    void* gauge[4] = {nullptr, nullptr, nullptr, nullptr};
    void* U_nat = nullptr;
    void* frag = nullptr;        // compact FP16 links for the matrix-core FP16 hop (4 | Ls)
    void* frag_b = nullptr;      // compact BF16 links for the matrix-core BF16 hop (4 | Ls)
    double* om = nullptr;
    std::vector<double> om_h;
    double* partial = nullptr;
    size_t npartial = 0;
    double* sc = nullptr;        // device scalar slots
    double* pinned = nullptr;    // host mirror of the slots
    double* ring = nullptr;      // pinned [2][4]: per-iteration scalars read one iteration late
    hipEvent_t ring_ev[2] = {nullptr, nullptr};
    std::map<std::string, Half> ws;
    std::map<std::string, void*> raw;
    // chronological guesses across solves (eofa_chrono): depth, solutions
    // stored per system (L, R) and the masses they were taken at
    int chrono_k = 0;
    int chrono_n[2] = {0, 0};
    double chrono_m[2][2] = {{0, 0}, {0, 0}};
    // timing
    bool timing = false;
    std::vector<hipEvent_t> evpool;
    std::vector<TimingRec> recs;
    long t_count[C_NCLS] = {0};
    double t_ms[C_NCLS] = {0}, t_bytes[C_NCLS] = {0};
    double flops = 0;
    bool use_mfma = true;
    int mfma_depth = 3;
};

namespace {

enum Slot { S_WW = 0, S_ZZ0 = 1, S_ZZ1 = 2, S_RR = 3, S_B2 = 4, S_T0 = 5, S_T1 = 6, S_ALPHA = 8,
            S_NSLOT = S_ALPHA + XBATCH };

size_t half_bytes(const eofa_ctx* c, int prec) { return (size_t)16 * nblocks_of(prec) * c->N; }

Half& ws(eofa_ctx* c, const std::string& name, int prec) {
    std::string key = name + "#" + std::to_string(prec);
    auto it = c->ws.find(key);
    if (it != c->ws.end()) return it->second;
    Half h;
    h.prec = prec;
    hipchk(hipMalloc(&h.d, half_bytes(c, prec)), "hipMalloc(field)");
    hipchk(hipMemsetAsync(h.d, 0, half_bytes(c, prec), c->st), "hipMemset(field)");
    if (prec == P16) {
        hipchk(hipMalloc((void**)&h.nrm, sizeof(float) * c->N), "hipMalloc(norm)");
        hipchk(hipMemsetAsync(h.nrm, 0, sizeof(float) * c->N, c->st), "hipMemset(norm)");
    }
    return c->ws[key] = h;
}

void* rawbuf(eofa_ctx* c, const std::string& name, size_t bytes) {
    auto it = c->raw.find(name);
    if (it != c->raw.end()) return it->second;
    void* p = nullptr;
    hipchk(hipMalloc(&p, bytes), "hipMalloc(buffer)");
    return c->raw[name] = p;
}

void* gauge_of(eofa_ctx* c, int prec) {
    if (!c->gauge[prec]) {
        const size_t nc = (size_t)2 * 8 * 9 * c->Vh;
        hipchk(hipMalloc(&c->gauge[prec], nc * complex_bytes(prec)), "hipMalloc(gauge)");
        hipchk(launch_gauge_convert(prec, c->gauge[P64], c->gauge[prec], nc, c->st), "gauge convert");
    }
    return c->gauge[prec];
}

// Block-major links of precision p's block table (FP32 links, or the compact
// 16-bit links of the matrix-core paths), rebuilt whenever the links change.
constexpr size_t link_record_bytes(int p) { return p == P64 ? 144 : p == P32 ? 72 : 36; }

void build_links_blocked(eofa_ctx* c, int p) {
    const void* src = p == P64 ? c->gauge[P64] : p == P32 ? gauge_of(c, P32) : (p == PB16 ? c->frag_b : c->frag);
    const int wide = p == P64 ? 2 : p == P32 ? 1 : 0;
    hipchk(launch_links_blocked(src, c->lnkb[p], c->sites[p], c->Vh, c->nblk_hop * c->NS, wide, c->st),
           "block-major links");
}

// ---- timing ---------------------------------------------------------------
int timing_begin(eofa_ctx* c) {
    if (!c->timing) return -1;
    const int idx = (int)c->recs.size() * 2;
    while ((int)c->evpool.size() < idx + 2) {
        hipEvent_t e;
        hipchk(hipEventCreate(&e), "hipEventCreate");
        c->evpool.push_back(e);
    }
    hipchk(hipEventRecord(c->evpool[idx], c->st), "hipEventRecord");
    return idx;
}

void timing_end(eofa_ctx* c, int idx, int cls, double bytes) {
    if (idx < 0) return;
    hipchk(hipEventRecord(c->evpool[idx + 1], c->st), "hipEventRecord");
    c->recs.push_back({cls, idx, bytes});
}

void timing_collect(eofa_ctx* c) {
    if (c->recs.empty()) return;
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    for (auto& r : c->recs) {
        float ms = 0;
        hipchk(hipEventElapsedTime(&ms, c->evpool[r.ev], c->evpool[r.ev + 1]), "hipEventElapsedTime");
        c->t_count[r.cls] += 1;
        c->t_ms[r.cls] += ms;
        c->t_bytes[r.cls] += r.bytes;
    }
    c->recs.clear();
}

// ---- operator pieces ---------------------------------------------------------
const Op5 I5{0, 0, 0.0, 0.0};
Op5 Dt(const eofa_ctx* c, int tr) { return Op5{1, tr, c->b5, c->c5}; }
Op5 DtInv(const eofa_ctx* c, int tr) { return Op5{2, tr, c->b5, c->c5}; }
Op5 Mee(const eofa_ctx* c, int tr) { return Op5{1, tr, c->beta0, c->beta1}; }
Op5 MeeInv(const eofa_ctx* c, int tr) { return Op5{2, tr, c->beta0, c->beta1}; }

// flops per 5D site: bidiagonal 72, inverse 144, dense block 48 Ls (24 reals x Ls multiply-adds)
double op_flops(const Op5& o, int Ls) {
    return o.kind == 1 ? 72.0 : o.kind == 2 ? 144.0 : o.kind == 3 ? 48.0 * Ls : 0.0;
}
// the dense blocks of D_EOFA's even-odd form (uploaded per mass pair by solve_dense)
Op5 D5(int tr) { return Op5{3, tr, 0.0, 0.0}; }
Op5 D5Inv(int tr) { return Op5{3, tr, 1.0, 0.0}; }

struct HopCall {
    int prec = P64;
    bool dag = false;
    bool hop = true;
    int par = 0;   // output parity
    const Half* in = nullptr;
    Half* out = nullptr;
    const Half* aux = nullptr;
    const Half* aux2 = nullptr;
    Op5 A = I5, B = I5, C = I5, B2 = I5;
    double ch = 1.0, ca = 1.0, cr = 1.0;
    double mp = 0, mm = 0;
    double* partial = nullptr;
    // ch and ca scaled on the device by sc[s_num] / sc[s_den] (saved to sc[s_alpha])
    bool dev_alpha = false;
    int s_num = 0, s_den = 0, s_alpha = -1;
    // dense blocks [D5+, D5-, D5inv+, D5inv-] (the dense D_EOFA path, any of its precisions)
    const double* dmat = nullptr;
};

void run_hop(eofa_ctx* c, const HopCall& h) {
    // epilogue forms the kernel implements: C(ch A(hop) + cr aux2) + ca B(aux) requires
    // C = 1 whenever aux is given, and aux2 only with A = 1 unless C = 1
    if (h.hop && h.aux && h.C.kind != 0) fail(EOFA_EDEVICE, "internal: aux with a non-trivial C");
    if (h.hop && h.aux2 && h.A.kind != 0 && h.C.kind != 0) fail(EOFA_EDEVICE, "internal: aux2 with A and C");
    if (!h.hop && h.aux2 && h.C.kind != 0) fail(EOFA_EDEVICE, "internal: aux2 after C");
    if (!h.hop && !h.aux) fail(EOFA_EDEVICE, "internal: local op without input");
    if (h.B2.kind != 0 && (!h.hop || !h.aux)) fail(EOFA_EDEVICE, "internal: B2 needs a hop with aux");
    HopArgs a;
    memset(&a, 0, sizeof(a));
    a.in = h.in ? h.in->d : nullptr;
    a.in_nrm = h.in ? h.in->nrm : nullptr;
    a.out = h.out->d;
    a.out_nrm = h.out->nrm;
    a.aux = h.aux ? h.aux->d : nullptr;
    a.aux_nrm = h.aux ? h.aux->nrm : nullptr;
    a.aux2 = h.aux2 ? h.aux2->d : nullptr;
    a.aux2_nrm = h.aux2 ? h.aux2->nrm : nullptr;
    a.nbr = c->nbr + (size_t)h.par * 8 * c->Vh;
    a.sites = c->sites[h.prec];
    a.par = h.par;
    const bool mfma = (h.prec == P16 || h.prec == PB16) && c->Ls % 4 == 0 && c->use_mfma;
    a.blk = (mfma || h.prec == P64 || h.prec == P32) && h.hop && c->blk[h.prec];
    if (a.blk) a.nbrb = c->nbrb[h.prec] + (size_t)h.par * 5 * c->nblk_hop * c->NS;
    if (h.hop && !mfma) {   // the matrix-core paths read only their compact 16-bit links
        const int lp = link_prec(h.prec);
        a.gauge = (const char*)gauge_of(c, lp) + (size_t)h.par * 8 * 9 * c->Vh * complex_bytes(lp);
    }
    if (h.hop && mfma) {
        const int bf = h.prec == PB16;
        void*& fr = bf ? c->frag_b : c->frag;
        if (!fr) {
            hipchk(hipMalloc(&fr, (size_t)2 * 8 * c->Vh * 36), "hipMalloc(16-bit links)");
            hipchk(launch_gauge_c16(c->gauge[P64], fr, c->Vh, bf, c->st), "16-bit links");
        }
        a.frag = (const char*)fr + (size_t)h.par * 8 * c->Vh * 36;
        a.depth = c->mfma_depth;
    }
    if (a.blk) {   // the block-sharing hops stage their links from the block-major copy
        const size_t per_par = (size_t)c->nblk_hop * c->NS * 8 * link_record_bytes(h.prec);
        if (!c->lnkb[h.prec]) {
            hipchk(hipMalloc(&c->lnkb[h.prec], 2 * per_par), "hipMalloc(block-major links)");
            build_links_blocked(c, h.prec);
        }
        a.lnkb = (const char*)c->lnkb[h.prec] + (size_t)h.par * per_par;
    }
    a.Vh = c->Vh;
    a.Ls = c->Ls;
    a.NS = c->NS;
    a.N = c->N;
    a.mp = h.mp;
    a.mm = h.mm;
    a.opA = h.A;
    a.opB = h.B;
    a.opC = h.C;
    a.opB2 = h.B2;
    a.ch = h.ch;
    a.ca = h.ca;
    a.cr = h.cr;
    a.partial = h.partial;
    if (h.dev_alpha) {
        a.dsc = c->sc;
        a.s_num = h.s_num;
        a.s_den = h.s_den;
        a.s_alpha = h.s_alpha;
    }
    // bookkeeping: flops (fixed convention) and algorithmic bytes
    double f = 0, nfields = 1;
    if (h.hop) f += 1320.0 + op_flops(h.A, c->Ls), nfields += 1;
    if (h.aux) f += op_flops(h.B, c->Ls) + op_flops(h.B2, c->Ls) + (h.hop ? 24.0 : 0.0), nfields += 1;
    if (h.aux2) f += 24.0, nfields += 1;
    f += op_flops(h.C, c->Ls);
    c->flops += f * (double)c->n5;
    double bytes = nfields * spinor_bytes(h.prec) * (double)c->n5;
    // algorithmic link bytes: the 4V links of one checkerboard hop, 9 complex
    // numbers each at the field precision (what the kernel reads can be more:
    // FP32 links or the FP16 rows of the matrix-core path)
    if (h.hop) bytes += 72.0 * complex_bytes(h.prec) * c->Vh;
    const int ev = timing_begin(c);
    if (h.dmat) {
        if ((h.prec != P64 && h.prec != P32 && h.prec != P16) || h.C.kind != 0 || h.B2.kind != 0 || h.dev_alpha)
            fail(EOFA_EDEVICE, "internal: unsupported dense hop form");
        // the dense hops run per site: where this precision's table lists
        // blocks they walk the per-site table instead (a block table spreads
        // each workgroup's slots over 8 rows)
        if (c->blk[h.prec]) a.sites = c->fsites;
        a.dmat = h.dmat;
        hipchk(launch_hop_dense(h.prec, h.dag, h.hop, a, c->nblk_hop, c->st), "dense hop kernel");
        timing_end(c, ev, h.hop ? C_HOPDENSE : C_BLAS, bytes);
        return;
    }
    if (h.A.kind == 3 || h.B.kind == 3) fail(EOFA_EDEVICE, "internal: dense block without matrices");
    hipchk(launch_hop(h.prec, h.dag, h.hop, a, c->nblk_hop, c->st), "hop kernel");
    timing_end(c, ev, h.hop ? (int)h.prec : C_BLAS, bytes);
}

// local 5D op: out = C(ca * B(aux))
void local_op(eofa_ctx* c, int prec, const Half& in, Half& out, Op5 B, Op5 C, double mp, double mm,
              double ca = 1.0) {
    HopCall h;
    h.prec = prec;
    h.hop = false;
    h.aux = &in;
    h.out = &out;
    h.B = B;
    h.C = C;
    h.ca = ca;
    h.mp = mp;
    h.mm = mm;
    run_hop(c, h);
}

void reduce(eofa_ctx* c, int n, int slot) {
    hipchk(launch_reduce(c->partial, n, c->sc, slot, c->st), "reduce");
}

double read_slot(eofa_ctx* c, int slot) {
    hipchk(hipMemcpyAsync(c->pinned + slot, c->sc + slot, sizeof(double), hipMemcpyDeviceToHost, c->st),
           "hipMemcpy(scalar)");
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    return c->pinned[slot];
}

// slots [first, first + n) to the host (one synchronisation)
const double* read_slots(eofa_ctx* c, int first, int n) {
    hipchk(hipMemcpyAsync(c->pinned + first, c->sc + first, sizeof(double) * n, hipMemcpyDeviceToHost, c->st),
           "hipMemcpy(scalars)");
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    return c->pinned + first;
}

double norm2(eofa_ctx* c, const Half& f, int slot) {
    hipchk(launch_norm2(f.prec, f.d, f.nrm, c->n5, c->N, c->partial, c->nblk_blas, c->st), "norm2");
    reduce(c, c->nblk_blas, slot);
    return read_slot(c, slot);
}

void convert(eofa_ctx* c, const Half& in, Half& out) {
    const int ev = timing_begin(c);
    hipchk(launch_convert(in.prec, out.prec, in.d, in.nrm, out.d, out.nrm, c->n5, c->N, c->nblk_blas, c->st),
           "convert");
    timing_end(c, ev, C_BLAS, (double)c->n5 * (spinor_bytes(in.prec) + spinor_bytes(out.prec)));
}

void zero(eofa_ctx* c, Half& f) {
    hipchk(launch_zero(f.prec, f.d, f.nrm, c->n5, c->N, c->nblk_blas, c->st), "zero");
}

// K1: tmp_e = M_ee^-1 Dtilde Dh_eo pt_o    (pt = Dtilde in)
void schur_k1(eofa_ctx* c, int prec, const Half& pt, Half& tmp, double mp, double mm) {
    HopCall h;
    h.prec = prec; h.par = 0; h.in = &pt; h.out = &tmp;
    h.A = Dt(c, 0); h.C = MeeInv(c, 0); h.mp = mp; h.mm = mm;
    run_hop(c, h);
}
// K2: out_o = M_ee p_o - Dh_oe tmp_e   (+ |out|^2 partials)
void schur_k2(eofa_ctx* c, int prec, const Half& tmp, const Half& p, Half& out, double mp, double mm,
              double* partial) {
    HopCall h;
    h.prec = prec; h.par = 1; h.in = &tmp; h.out = &out; h.ch = -1.0;
    h.aux = &p; h.B = Mee(c, 0); h.ca = 1.0; h.mp = mp; h.mm = mm; h.partial = partial;
    run_hop(c, h);
}
// K2 for a direction kept as pt = Dtilde p:  out_o = M_ee Dtilde^-1 pt_o - Dh_oe tmp_e
void schur_k2_tilde(eofa_ctx* c, int prec, const Half& tmp, const Half& pt, Half& out, double mp, double mm,
                    double* partial) {
    HopCall h;
    h.prec = prec; h.par = 1; h.in = &tmp; h.out = &out; h.ch = -1.0;
    h.aux = &pt; h.B = Mee(c, 0); h.B2 = DtInv(c, 0); h.ca = 1.0; h.mp = mp; h.mm = mm; h.partial = partial;
    run_hop(c, h);
}
// K3: tmp_e = M_ee^-dag Dtilde^dag Dh^dag_eo in_o
void schur_k3(eofa_ctx* c, int prec, const Half& in, Half& tmp, double mp, double mm) {
    HopCall h;
    h.prec = prec; h.dag = true; h.par = 0; h.in = &in; h.out = &tmp;
    h.A = Dt(c, 1); h.C = MeeInv(c, 1); h.mp = mp; h.mm = mm;
    run_hop(c, h);
}
// K4: out_o = M_ee^dag in_o - Dtilde^dag Dh^dag_oe tmp_e   (+ partials)
void schur_k4(eofa_ctx* c, int prec, const Half& tmp, const Half& in, Half& out, double mp, double mm,
              double* partial) {
    HopCall h;
    h.prec = prec; h.dag = true; h.par = 1; h.in = &tmp; h.out = &out; h.A = Dt(c, 1); h.ch = -1.0;
    h.aux = &in; h.B = Mee(c, 1); h.ca = 1.0; h.mp = mp; h.mm = mm; h.partial = partial;
    run_hop(c, h);
}

// K4 with the CG update folded in:
//   z <- z - alpha Mhat^dag w = z - alpha M_ee^dag w + alpha Dtilde^dag Dh^dag_oe tmp_e,
// alpha = sc[s_num] / sc[s_den] read on the device and saved to sc[s_alpha]  (+ |z|^2 partials)
void schur_k4_update(eofa_ctx* c, int prec, const Half& tmp, const Half& w, Half& z, double mp, double mm,
                     int s_num, int s_den, int s_alpha, double* partial) {
    HopCall h;
    h.prec = prec; h.dag = true; h.par = 1; h.in = &tmp; h.out = &z; h.A = Dt(c, 1); h.ch = 1.0;
    h.aux = &w; h.B = Mee(c, 1); h.ca = -1.0; h.aux2 = &z; h.cr = 1.0; h.mp = mp; h.mm = mm;
    h.partial = partial;
    h.dev_alpha = true; h.s_num = s_num; h.s_den = s_den; h.s_alpha = s_alpha;
    run_hop(c, h);
}

// p <- z + beta p_old (or p <- z), pt <- Dtilde p; beta = sc[i_new] / sc[i_old]
// (pt == nullptr: p <- Dtilde z + beta p, the direction kept in Cayley form)
void pupdate(eofa_ctx* c, int prec, const Half& z, const Half* pold, Half& p, Half* pt, int i_new, int i_old,
             double mp, double mm) {
    const int ev = timing_begin(c);
    hipchk(launch_pupdate(prec, z.d, z.nrm, pold ? pold->d : nullptr, pold ? pold->nrm : nullptr, p.d, p.nrm,
                          pt ? pt->d : nullptr, pt ? pt->nrm : nullptr, c->sc, i_new, i_old, pold ? 0 : 1, c->Vh,
                          c->Ls, c->NS, c->N, c->b5, c->c5, mp, mm, c->nblk_hop, c->st),
           "pupdate");
    timing_end(c, ev, C_BLAS, (double)c->n5 * ((pold ? 3.0 : 2.0) + (pt ? 1.0 : 0.0)) * spinor_bytes(prec));
}

void check_finite(double v, const char* what) {
    if (!std::isfinite(v)) fail(EOFA_ENAN, std::string("non-finite ") + what);
}

struct SolveResult {
    int iters = 0;
    int reliable = 0;
    bool converged = false;
    bool stagnated = false;   // the inner precision stopped making progress (mixed only)
};

// Solve Mhat x_o = bhat_o by CGNR, x_o holding the initial guess.
// Stops when |bhat - Mhat x| <= thresh.  prec == P64 without `fused`: plain
// FP64 CGNR.  Otherwise the reliable-update iteration with inner precision
// `prec` (with prec == P64 and `fused`: the same iteration, every step in
// FP64, so that it differs from the plain CGNR only by its fusions).
SolveResult cgnr_schur(eofa_ctx* c, double mp, double mm, const Half& bhat, Half& x, bool guess,
                       double thresh, int maxiter, int prec, double delta, bool fused = false) {
    SolveResult res;
    const int nb = c->nblk_hop;
    Half& tmp64 = ws(c, "tmp_e", P64);
    Half& r64 = ws(c, "r", P64);
    Half& xt64 = ws(c, "xt", P64);
    // r = bhat - Mhat x
    auto true_residual = [&](void) -> double {
        HopCall h;
        local_op(c, P64, x, xt64, Dt(c, 0), I5, mp, mm);
        schur_k1(c, P64, xt64, tmp64, mp, mm);
        h.prec = P64; h.par = 1; h.in = &tmp64; h.out = &r64; h.ch = 1.0;
        h.aux = &x; h.B = Mee(c, 0); h.ca = -1.0; h.aux2 = &bhat; h.cr = 1.0;
        h.mp = mp; h.mm = mm; h.partial = c->partial;
        run_hop(c, h);
        reduce(c, nb, S_RR);
        return read_slot(c, S_RR);
    };
    double rr;
    if (guess) {
        rr = true_residual();
    } else {
        zero(c, x);
        convert(c, bhat, r64);
        rr = norm2(c, r64, S_RR);
    }
    check_finite(rr, "residual norm");
    if (std::sqrt(rr) <= thresh) { res.converged = true; return res; }

    const bool mixed = prec != P64 || fused;
    const int px = prec != P64 ? P32 : P64;
    Half& r = mixed ? ws(c, "r_lo", prec) : r64;
    Half& z = ws(c, "z", prec);
    Half* pr[XBATCH];   // ring of search directions p_k (buffer k mod XBATCH)
    for (int j = 0; j < XBATCH; ++j) pr[j] = &ws(c, "p" + std::to_string(j), prec);
    Half* ptp = mixed ? nullptr : &ws(c, "pt", prec);   // Dtilde p (FP64 path)
    Half& w = ws(c, "w", prec);
    Half& tmp = ws(c, "tmp_lo_e", prec);
    Half& xl = mixed ? ws(c, "x_lo", px) : x;
    if (mixed) {
        convert(c, r64, r);
        zero(c, xl);
    }
    // x += sum alpha_j p_j for the pending directions [pending0, k]
    int pending0 = 0;
    auto flush = [&](int k) {
        const int cnt = k - pending0 + 1;
        if (cnt <= 0) return;
        const void* pp[XBATCH];
        const float* pn[XBATCH];
        int sl[XBATCH];
        for (int j = 0; j < cnt; ++j) {
            const int it = pending0 + j;
            pp[j] = pr[it % XBATCH]->d;
            pn[j] = pr[it % XBATCH]->nrm;
            sl[j] = S_ALPHA + it % XBATCH;
        }
        const int ev = timing_begin(c);
        hipchk(launch_x_batch(prec, xl.d, xl.nrm, pp, pn, sl, cnt, c->sc, c->n5, c->N, c->nblk_blas, c->st),
               "x update");
        timing_end(c, ev, C_BLAS, (double)c->n5 * (2.0 * spinor_bytes(px) + cnt * spinor_bytes(prec)));
        c->flops += 48.0 * cnt * (double)c->n5;
        pending0 = k + 1;
    };
    int cur = S_ZZ0, nxt = S_ZZ1;
    // z = Mhat^dag r ; p_0 = z ; pt = Dtilde p_0 (mixed: the ring holds Dtilde p)
    schur_k3(c, prec, r, tmp, mp, mm);
    schur_k4(c, prec, tmp, r, z, mp, mm, c->partial);
    reduce(c, nb, cur);
    pupdate(c, prec, z, nullptr, *pr[0], ptp, cur, cur, mp, mm);
    double rmax = std::sqrt(rr);
    int k = 0;
    if (mixed) {
        // The search directions are kept in Cayley form, pt_k = Dtilde p_k:
        // K1 reads pt_k, K2 forms M_ee p_k = M_ee Dtilde^-1 pt_k in its
        // epilogue, and x_lo accumulates Dtilde x (undone before each
        // reliable update), which saves writing p next to pt.
        auto fold_x = [&]() {
            local_op(c, px, xl, xl, I5, DtInv(c, 0), mp, mm);
            hipchk(launch_accum_hi(px, x.d, xl.d, xl.nrm, c->n5, c->N, c->nblk_blas, c->st), "accum");
        };
        // Low-precision iterations keep z = Mhat^dag r by its own recursion
        // z <- z - alpha Mhat^dag w (folded into K4, so r is not stored);
        // |r|^2 follows |r_{k+1}|^2 = |r_k|^2 - alpha |z_k|^2 (exact in exact
        // arithmetic, since (r_k, Mhat p_k) = (z_k, p_k) = |z_k|^2).  Reliable
        // updates replace the estimate by the FP64 true residual and z by
        // Mhat^dag of it; convergence is only declared on a true residual.
        // The scalars of iteration k are copied to the host ring after its K4
        // and read while iteration k+1 runs, so the host never waits on an
        // idle GPU; decisions therefore use the estimate one iteration late.
        double rr_est = rr;
        int pend_cur = -1;          // slot of |z_k|^2 of the pending ring entry, -1: none
        // Stagnation guard: in 16-bit arithmetic the recursion can stall
        // (lost conjugacy) with the estimate above delta |r|.  A segment
        // longer than max(400, 4 x the longest one so far) forces a reliable
        // update and restarts the directions from z.
        int seg_iters = 0, seg_max = 0;
        // Progress check: a healthy solve halves the true residual every few
        // dozen iterations.  1000 iterations without halving it force a
        // reliable update; if that confirms it, the inner precision is
        // exhausted and the caller continues one precision up.
        double r_halve = rmax;
        int it_halve = res.iters;
        while (res.iters < maxiter) {
            Half& p = *pr[k % XBATCH];
            schur_k1(c, prec, p, tmp, mp, mm);
            schur_k2_tilde(c, prec, tmp, p, w, mp, mm, c->partial);
            reduce(c, nb, S_WW);
            schur_k3(c, prec, w, tmp, mp, mm);
            schur_k4_update(c, prec, tmp, w, z, mp, mm, cur, S_WW, S_ALPHA + k % XBATCH, c->partial);
            reduce(c, nb, nxt);
            res.iters++;
            double* slot_k = c->ring + 4 * (k & 1);
            hipchk(hipMemcpyAsync(slot_k, c->sc + S_WW, sizeof(double) * 3, hipMemcpyDeviceToHost, c->st),
                   "hipMemcpy(scalars)");
            hipchk(hipEventRecord(c->ring_ev[k & 1], c->st), "hipEventRecord");
            if (pend_cur >= 0) {   // iteration k-1
                hipchk(hipEventSynchronize(c->ring_ev[(k - 1) & 1]), "hipEventSynchronize");
                const double* sv = c->ring + 4 * ((k - 1) & 1);
                const double ww = sv[0], zz = sv[pend_cur - S_WW], zn = sv[(pend_cur == S_ZZ0 ? S_ZZ1 : S_ZZ0) - S_WW];
                check_finite(ww, "|Mhat p|^2");
                check_finite(zn, "|z|^2");
                rr_est -= zz / ww * zz;
            }
            pend_cur = cur;
            const double rn = std::sqrt(std::max(rr_est, 0.0));
            ++seg_iters;
            const bool stalled = seg_iters > std::max(400, 4 * seg_max);
            const bool overdue = res.iters - it_halve > 1000;
            bool restart = false;
            if (rn <= delta * rmax || rn <= thresh || stalled || overdue) {
                // reliable update: fold the directions into x_lo, x_lo into x, recompute r in FP64
                flush(k);
                fold_x();
                rr = true_residual();
                check_finite(rr, "true residual");
                res.reliable++;
                const double rprev = rmax;
                rmax = std::sqrt(rr);
                rr_est = rr;
                pend_cur = -1;   // the true residual includes iteration k
                seg_max = std::max(seg_max, seg_iters);
                seg_iters = 0;
                restart = stalled;
                if (rmax <= thresh) { res.converged = true; break; }
                if (rmax <= 0.5 * r_halve) {
                    r_halve = rmax;
                    it_halve = res.iters;
                }
                // a stalled segment (over 400 iterations) that did not even halve
                // the true residual, or 1000 iterations without halving it: the
                // inner precision is exhausted here
                if ((stalled && rmax > 0.5 * rprev) || res.iters - it_halve > 1000) {
                    res.stagnated = true;
                    break;
                }
                convert(c, r64, r);
                schur_k3(c, prec, r, tmp, mp, mm);
                schur_k4(c, prec, tmp, r, z, mp, mm, c->partial);
                reduce(c, nb, nxt);
            }
            if (k - pending0 + 1 == XBATCH) flush(k);
            if (res.iters >= maxiter) { flush(k); break; }
            Half& pn1 = *pr[(k + 1) % XBATCH];
            pupdate(c, prec, z, restart ? nullptr : &p, pn1, nullptr, nxt, cur, mp, mm);
            c->flops += 72.0 * (double)c->n5 + 48.0 * (double)c->n5;
            std::swap(cur, nxt);
            ++k;
        }
        if (!res.converged) fold_x();
        return res;
    }
    // FP64: plain CGNR with the recursively updated residual r
    Half& pt = *ptp;
    while (res.iters < maxiter) {
        Half& p = *pr[k % XBATCH];
        // w = Mhat p, |w|^2
        schur_k1(c, prec, pt, tmp, mp, mm);
        schur_k2(c, prec, tmp, p, w, mp, mm, c->partial);
        reduce(c, nb, S_WW);
        // r -= alpha w, |r|^2 (alpha kept for the batched x update)
        {
            const int ev = timing_begin(c);
            hipchk(launch_r_update(prec, r.d, r.nrm, w.d, w.nrm, c->sc, cur, S_WW, S_ALPHA + k % XBATCH,
                                   c->n5, c->N, c->partial, c->nblk_blas, c->st), "r update");
            timing_end(c, ev, C_BLAS, (double)c->n5 * 3.0 * spinor_bytes(prec));
            c->flops += 48.0 * (double)c->n5;
        }
        reduce(c, c->nblk_blas, S_RR);
        res.iters++;
        rr = read_slot(c, S_RR);
        check_finite(rr, "residual norm");
        if (std::sqrt(rr) <= thresh) {
            flush(k);
            res.converged = true;
            break;
        }
        if (k - pending0 + 1 == XBATCH) flush(k);
        if (res.iters >= maxiter) { flush(k); break; }
        // z = Mhat^dag r, |z|^2 ; p_{k+1} = z + beta p_k ; pt = Dtilde p_{k+1}
        schur_k3(c, prec, r, tmp, mp, mm);
        schur_k4(c, prec, tmp, r, z, mp, mm, c->partial);
        reduce(c, nb, nxt);
        Half& pn1 = *pr[(k + 1) % XBATCH];
        pupdate(c, prec, z, &p, pn1, &pt, nxt, cur, mp, mm);
        c->flops += 72.0 * (double)c->n5 + 48.0 * (double)c->n5;
        std::swap(cur, nxt);
        ++k;
    }
    return res;
}

struct CayleyOut {
    int iters = 0, reliable = 0;
    double true_resid = 0;
    bool converged = false;
    int inner_used = P64;   // the most precise inner arithmetic used (after escalations)
};

void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Z);

// Earlier odd-site solutions y_i (FP64) and room for Mhat y_i, for the
// chronological initial guess of Section 5.2.
struct Forecast {
    Half* const* y;
    Half* const* w;
    int k;
};

// <a, b> over FP64 half fields (deterministic two-stage reduction)
void cdot64(eofa_ctx* c, const Half& a, const Half& b, double* re, double* im) {
    const int nb = c->nblk_blas;
    hipchk(launch_cdot64(a.d, b.d, c->n5, c->N, c->partial, nb, c->st), "cdot");
    hipchk(launch_reduce(c->partial, nb, c->sc, S_T0, c->st), "reduce");
    hipchk(launch_reduce(c->partial + nb, nb, c->sc, S_T1, c->st), "reduce");
    const double* v = read_slots(c, S_T0, 2);
    *re = v[0];
    *im = v[1];
    check_finite(*re + *im, "forecast inner product");
}

// Chronological guess (Brower et al.): yo = sum_i c_i y_i minimising
// |bhat - Mhat yo| over the span of the earlier solutions, which for CGNR is
// also the minimum of the Mhat^dag Mhat energy norm of the error.  The
// normal equations G c = h, G_ij = <Mhat y_i, Mhat y_j>, h_i = <Mhat y_i, bhat>,
// are solved on the host through the real symmetric form of G with
// eigenvalues below 1e-12 of the largest dropped (the y_i are close to
// linearly dependent).
void forecast_guess(eofa_ctx* c, double mp, double mm, const Half& bhat, const Forecast& f, Half& yo) {
    const int k = f.k;
    Half& te = ws(c, "fc_t_e", P64);
    Half& to = ws(c, "fc_t_o", P64);
    for (int i = 0; i < k; ++i) {
        local_op(c, P64, *f.y[i], to, Dt(c, 0), I5, mp, mm);
        schur_k1(c, P64, to, te, mp, mm);
        schur_k2(c, P64, te, *f.y[i], *f.w[i], mp, mm, nullptr);
    }
    const int n = 2 * k;
    std::vector<double> A((size_t)n * n), rhs(n), Z;
    for (int i = 0; i < k; ++i) {
        for (int j = i; j < k; ++j) {
            double gr, gi;
            cdot64(c, *f.w[i], *f.w[j], &gr, &gi);
            // [[Re G, -Im G], [Im G, Re G]] with G_ji = conj(G_ij)
            A[(size_t)i * n + j] = A[(size_t)(k + i) * n + (k + j)] = gr;
            A[(size_t)j * n + i] = A[(size_t)(k + j) * n + (k + i)] = gr;
            A[(size_t)(k + i) * n + j] = gi;
            A[(size_t)i * n + (k + j)] = -gi;
            A[(size_t)(k + j) * n + i] = -gi;
            A[(size_t)j * n + (k + i)] = gi;
        }
        double hr, hi;
        cdot64(c, *f.w[i], bhat, &hr, &hi);
        rhs[i] = hr;
        rhs[k + i] = hi;
    }
    jacobi_eigen(n, A, Z);
    double lmax = 0;
    for (int j = 0; j < n; ++j) lmax = std::max(lmax, A[(size_t)j * n + j]);
    std::vector<double> x(n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double lam = A[(size_t)j * n + j];
        if (!(lam > 1e-12 * lmax)) continue;
        double d = 0;
        for (int r = 0; r < n; ++r) d += Z[(size_t)r * n + j] * rhs[r];
        for (int r = 0; r < n; ++r) x[r] += Z[(size_t)r * n + j] * d / lam;
    }
    zero(c, yo);
    for (int i = 0; i < k; ++i)
        hipchk(launch_caxpy64(yo.d, f.y[i]->d, x[i], x[k + i], c->n5, c->N, c->nblk_blas, c->st), "caxpy");
}

// Solve D_DWF(mp, mm) y = b (even-odd, Section 5.1), then chi = Dtilde y.
// y_e/y_o hold an initial guess when `guess`.  Writes chi_e/chi_o.
CayleyOut solve_cayley(eofa_ctx* c, double mp, double mm, const Half& be, const Half& bo, Half& ye,
                       Half& yo, bool guess, Half& chie, Half& chio, const eofa_solver_t& sp,
                       const Forecast* fc = nullptr) {
    CayleyOut out;
    const int nb = c->nblk_hop;
    // |b|^2
    const double b2 = norm2(c, be, S_B2) + norm2(c, bo, S_B2);
    check_finite(b2, "source norm");
    if (b2 == 0.0) {
        zero(c, ye); zero(c, yo); zero(c, chie); zero(c, chio);
        out.converged = true;
        return out;
    }
    const double bnorm = std::sqrt(b2);
    // bhat_o = b_o - Dh_oe Dtilde M_ee^-1 b_e
    Half& t = ws(c, "t_e", P64);
    Half& bhat = ws(c, "bhat", P64);
    local_op(c, P64, be, t, Dt(c, 0), MeeInv(c, 0), mp, mm);
    {
        HopCall h;
        h.prec = P64; h.par = 1; h.in = &t; h.out = &bhat; h.ch = -1.0;
        h.aux2 = &bo; h.cr = 1.0; h.mp = mp; h.mm = mm;
        run_hop(c, h);
    }
    int prec = sp.inner;
    bool fused = prec == P64 && sp.fused_fp64 != 0;
    out.inner_used = prec;
    double thresh = 0.5 * sp.tol * bnorm;
    bool have = guess;
    if (fc && fc->k > 0) {   // chronological guess from earlier solutions (Section 5.2)
        forecast_guess(c, mp, mm, bhat, *fc, yo);
        have = true;
    }
    for (int attempt = 0; attempt < 6; ++attempt) {
        SolveResult r = cgnr_schur(c, mp, mm, bhat, yo, have, thresh, sp.maxiter - out.iters, prec,
                                   sp.reliable_delta > 0 ? sp.reliable_delta : 0.1, fused);
        out.iters += r.iters;
        out.reliable += r.reliable;
        // y_e = M_ee^-1 (b_e - Dh_eo Dtilde y_o)
        Half& yt = ws(c, "xt", P64);
        local_op(c, P64, yo, yt, Dt(c, 0), I5, mp, mm);
        {
            HopCall h;
            h.prec = P64; h.par = 0; h.in = &yt; h.out = &ye; h.ch = -1.0;
            h.aux2 = &be; h.cr = 1.0; h.C = MeeInv(c, 0); h.mp = mp; h.mm = mm;
            run_hop(c, h);
        }
        // chi = Dtilde y
        local_op(c, P64, ye, chie, Dt(c, 0), I5, mp, mm);
        local_op(c, P64, yo, chio, Dt(c, 0), I5, mp, mm);
        // true residual of the full system: b_p - M_ee y_p - Dh (Dtilde y)_pbar
        Half& rt = ws(c, "rt", P64);
        for (int par = 0; par < 2; ++par) {
            HopCall h;
            h.prec = P64; h.par = par; h.in = par ? &chie : &chio; h.out = &rt; h.ch = -1.0;
            h.aux = par ? &yo : &ye; h.B = Mee(c, 0); h.ca = -1.0;
            h.aux2 = par ? &bo : &be; h.cr = 1.0; h.mp = mp; h.mm = mm;
            h.partial = c->partial + (size_t)par * nb;
            run_hop(c, h);
        }
        reduce(c, 2 * nb, S_T0);
        const double rr = read_slot(c, S_T0);
        check_finite(rr, "true residual");
        out.true_resid = std::sqrt(rr) / bnorm;
        out.converged = out.true_resid <= sp.tol;
        if (out.converged || out.iters >= sp.maxiter) break;
        if (r.stagnated) {   // continue from y one precision up: 16-bit -> FP32 -> FP64
            if (prec == P64) fused = false;   // fused FP64 stalled: the plain CGNR takes over
            else prec = prec == P32 ? P64 : P32;
            out.inner_used = prec;
            have = true;
            continue;
        }
        if (!r.converged) break;
        // the recursively updated residual drifted: tighten and continue from y
        thresh *= 0.25 * sp.tol / out.true_resid;
        have = true;
    }
    return out;
}

void validate_solver(const eofa_solver_t* sp);
void omega_k(const eofa_ctx* c, double m1, double m2, double* k);

// ---- the dense D_EOFA comparison path (Table 4, "EOFA (dense)") --------------
// D_EOFA = D_DWF Dtilde^-1 = D_w + (1 - L) Dtilde^-1: the Wilson hop, diagonal
// in s, plus the site-local D5 = (4 - M5) + (1 - L) Dtilde^-1, dense in s (one
// Ls x Ls block per chirality).  Without the Cayley-form right
// preconditioning the EOFA systems D_EOFA chi = b are solved as they stand:
// even-odd, Mhat = D5 - Dh_oe D5^-1 Dh_eo on odd sites, FP64 CGNR.  Since
// D_DWF = D_EOFA Dtilde, b - D_EOFA chi is exactly the residual b - D_DWF y of
// the Cayley-form solve (chi = Dtilde y), so the two paths stop on the same
// quantity.

// in-place inverse of a row-major n x n matrix, Gauss-Jordan with partial pivoting
void invert_dense(int n, std::vector<double>& A) {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
        const double d = A[(size_t)piv * n + col];
        if (!(std::fabs(d) > 0.0) || !std::isfinite(d)) fail(EOFA_EINVAL, "singular 5D block of D_EOFA");
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)piv * n + k], A[(size_t)col * n + k]);
                std::swap(I[(size_t)piv * n + k], I[(size_t)col * n + k]);
            }
        for (int k = 0; k < n; ++k) {
            A[(size_t)col * n + k] /= d;
            I[(size_t)col * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
                I[(size_t)r * n + k] -= f * I[(size_t)col * n + k];
            }
        }
    }
    A.swap(I);
}

// [D5+, D5-, D5inv+, D5inv-] for boundary masses (m+, m-), each Ls x Ls row
// major, with L+ (m+) acting on spins 0, 1 and L- (m-) on spins 2, 3
std::vector<double> dense_blocks(const eofa_ctx* c, double mp, double mm) {
    const int n = c->Ls;
    const size_t nn = (size_t)n * n;
    std::vector<double> out(4 * nn);
    for (int ch = 0; ch < 2; ++ch) {
        const double m = ch == 0 ? mp : mm;
        std::vector<double> L(nn, 0.0);
        for (int s = 0; s < n; ++s) {
            if (ch == 0) {   // (L+ v)_s = v_{s-1}, (L+ v)_0 = -m+ v_{Ls-1}
                if (s >= 1) L[(size_t)s * n + s - 1] += 1.0;
                else L[(size_t)n - 1] += -m;
            } else {         // (L- v)_s = v_{s+1}, (L- v)_{Ls-1} = -m- v_0
                if (s <= n - 2) L[(size_t)s * n + s + 1] += 1.0;
                else L[(size_t)(n - 1) * n] += -m;
            }
        }
        std::vector<double> Dti(nn);
        for (size_t q = 0; q < nn; ++q) Dti[q] = c->c5 * L[q];
        for (int i = 0; i < n; ++i) Dti[(size_t)i * n + i] += c->b5;
        invert_dense(n, Dti);
        std::vector<double> D((nn));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = Dti[(size_t)i * n + j] + (i == j ? 4.0 - c->M5 : 0.0);
                for (int k = 0; k < n; ++k) v -= L[(size_t)i * n + k] * Dti[(size_t)k * n + j];
                D[(size_t)i * n + j] = v;
            }
        std::copy(D.begin(), D.end(), out.begin() + ch * nn);
        invert_dense(n, D);
        std::copy(D.begin(), D.end(), out.begin() + (2 + ch) * nn);
    }
    return out;
}

struct DenseOut {
    int iters = 0;
    int reliable = 0;
    double true_resid = 0;
    bool converged = false;
    int inner_used = P64;   // the most precise inner arithmetic used (after escalations)
};

// Dense hop forms in precision prec: out = ch DA(Dh in) + ca DB(aux) + cr aux2 on output parity par
void dense_hop(eofa_ctx* c, const double* dm, int prec, bool dag, int par, const Half* in, Half& out, Op5 A,
               double ch, const Half* aux, Op5 B, double ca, const Half* aux2, double cr, double* partial) {
    HopCall h;
    h.prec = prec; h.dag = dag; h.hop = in != nullptr; h.par = par; h.in = in; h.out = &out;
    h.A = A; h.ch = ch; h.aux = aux; h.B = B; h.ca = ca; h.aux2 = aux2; h.cr = cr;
    h.partial = partial; h.dmat = dm;
    run_hop(c, h);
}

// Even-odd CGNR on Mhat = D5 - Dh_oe D5^-1 Dh_eo.  sp.inner = FP64: plain
// CGNR.  FP32 or FP16 (+ site norm): the same recursion in that storage with
// FP32 arithmetic (x summed in FP32) and reliable updates, as in the
// Cayley-form solver: when
// the recursive |s| falls below delta times the true residual of the last
// update, x is folded into the FP64 solution and s = bhat - Mhat x is
// recomputed in FP64.
DenseOut solve_dense(eofa_ctx* c, const double* dm, const Half& be, const Half& bo, Half& xe, Half& xo,
                     const eofa_solver_t& sp) {
    DenseOut out;
    const int nb = c->nblk_hop;
    const double b2 = norm2(c, be, S_B2) + norm2(c, bo, S_B2);
    check_finite(b2, "source norm");
    if (b2 == 0.0) {
        zero(c, xe); zero(c, xo);
        out.converged = true;
        return out;
    }
    const double bnorm = std::sqrt(b2);
    int prec = sp.inner == EOFA_FP32 ? P32 : sp.inner == EOFA_FP16 ? P16 : P64;
    out.inner_used = prec;
    Half& t64 = ws(c, "dn_t", P64);
    Half& bh = ws(c, "dn_bhat", P64);
    Half& s64 = ws(c, "dn_s", P64);
    // bhat_o = b_o - Dh_oe D5^-1 b_e
    dense_hop(c, dm, P64, false, 0, nullptr, t64, I5, 1.0, &be, D5Inv(0), 1.0, nullptr, 0.0, nullptr);
    dense_hop(c, dm, P64, false, 1, &t64, bh, I5, -1.0, nullptr, I5, 0.0, &bo, 1.0, nullptr);
    zero(c, xo);
    const double target = sp.tol * bnorm;
    const double delta = sp.reliable_delta > 0 ? sp.reliable_delta : 0.1;
    // s64 = bhat - Mhat x_o in FP64 (Mhat x = D5 x - Dh_oe D5^-1 Dh_eo x), |s64|^2 in slot S_T1
    auto true_residual = [&]() -> double {
        dense_hop(c, dm, P64, false, 0, &xo, t64, D5Inv(0), 1.0, nullptr, I5, 0.0, nullptr, 0.0, nullptr);
        dense_hop(c, dm, P64, false, 1, &t64, s64, I5, 1.0, &xo, D5(0), -1.0, &bh, 1.0, c->partial);
        reduce(c, nb, S_T1);
        const double rr = read_slot(c, S_T1);
        check_finite(rr, "true residual");
        return std::sqrt(rr);
    };
    // The CG runs in `prec` from the current x_o.  A 16-bit (then FP32)
    // solve that stops making progress continues one precision up from its
    // iterate, as in the Cayley-form solver: the reduced-precision recursion
    // can stall (lost conjugacy) with its residual estimate above the
    // reliable-update threshold.
    for (int attempt = 0; attempt < 3; ++attempt) {
        const bool mixed = prec != P64;
        Half& t = ws(c, "dn_t", prec);
        Half& sr = ws(c, "dn_s", prec);   // s = bhat - Mhat x_o (its recursion)
        Half& r = ws(c, "dn_r", prec);    // r = Mhat^dag s
        Half& p = ws(c, "dn_p", prec);
        Half& w = ws(c, "dn_w", prec);
        Half& xl = mixed ? ws(c, "dn_xlo", P32) : xo;   // where the iterations sum x
        auto mhat = [&](const Half& in, Half& o, double* partial) {   // o = Mhat in
            dense_hop(c, dm, prec, false, 0, &in, t, D5Inv(0), 1.0, nullptr, I5, 0.0, nullptr, 0.0, nullptr);
            dense_hop(c, dm, prec, false, 1, &t, o, I5, -1.0, &in, D5(0), 1.0, nullptr, 0.0, partial);
        };
        auto mhat_dag = [&](const Half& in, Half& o, double* partial) {   // o = Mhat^dag in
            dense_hop(c, dm, prec, true, 0, &in, t, D5Inv(1), 1.0, nullptr, I5, 0.0, nullptr, 0.0, nullptr);
            dense_hop(c, dm, prec, true, 1, &t, o, I5, -1.0, &in, D5(1), 1.0, nullptr, 0.0, partial);
        };
        auto fold = [&]() {   // x_o += x_lo, x_lo = 0
            hipchk(launch_accum_hi(P32, xo.d, xl.d, xl.nrm, c->n5, c->N, c->nblk_blas, c->st), "accum");
        };
        if (mixed) zero(c, xl);
        double rmax;   // true residual at the last reliable update
        if (attempt == 0) {
            convert(c, bh, sr);
            rmax = std::sqrt(norm2(c, bh, S_T1));
        } else {
            rmax = true_residual();
            convert(c, s64, sr);
        }
        if (rmax <= target) break;
        // p = r = Mhat^dag s
        auto restart = [&]() -> double {
            mhat_dag(sr, r, c->partial);
            reduce(c, nb, S_T0);
            const double g = read_slot(c, S_T0);
            check_finite(g, "dense CG");
            convert(c, r, p);
            return g;
        };
        double gam = restart();
        // progress guard (mixed only): a segment between reliable updates
        // longer than max(400, 4 x the longest so far), or 1000 iterations
        // without halving the true residual, forces a reliable update; if
        // that confirms the stall, this precision is exhausted
        int seg_iters = 0, seg_max = 0, it_halve = out.iters;
        double r_halve = rmax;
        bool stagnated = false;
        while (out.iters < sp.maxiter && gam > 0.0) {
            mhat(p, w, c->partial);
            reduce(c, nb, S_T0);
            const double ww = read_slot(c, S_T0);
            check_finite(ww, "dense CG");
            if (!(ww > 0.0)) break;
            const double alpha = gam / ww;
            // x += alpha p ; s -= alpha w ; |s|^2
            const int ev = timing_begin(c);
            hipchk(launch_cg_step(prec, xl.d, p.d, p.nrm, sr.d, sr.nrm, w.d, w.nrm, alpha, c->n5, c->N,
                                  c->partial, c->nblk_blas, c->st),
                   "cg step");
            timing_end(c, ev, C_BLAS, (double)c->n5 * 6.0 * spinor_bytes(prec));
            reduce(c, c->nblk_blas, S_T1);
            ++out.iters;
            ++seg_iters;
            double rn = std::sqrt(read_slot(c, S_T1));
            check_finite(rn, "dense CG");
            const bool stalled = mixed && seg_iters > std::max(400, 4 * seg_max);
            const bool overdue = mixed && out.iters - it_halve > 1000;
            if (mixed && (rn <= delta * rmax || rn <= target || stalled || overdue)) {
                // reliable update: s = bhat - Mhat x in FP64
                fold();
                const double rprev = rmax;
                rmax = rn = true_residual();
                ++out.reliable;
                convert(c, s64, sr);
                seg_max = std::max(seg_max, seg_iters);
                seg_iters = 0;
                if (rn <= target) break;
                if (rmax <= 0.5 * r_halve) {
                    r_halve = rmax;
                    it_halve = out.iters;
                }
                if ((stalled && rmax > 0.5 * rprev) || out.iters - it_halve > 1000) {
                    stagnated = true;
                    break;
                }
                if (stalled) {   // lost conjugacy: restart the directions from the true residual
                    gam = restart();
                    continue;
                }
            }
            if (rn <= target) break;
            mhat_dag(sr, r, c->partial);
            reduce(c, nb, S_T0);
            const double g2 = read_slot(c, S_T0);
            check_finite(g2, "dense CG");
            // p <- r + (g2 / gam) p
            dense_hop(c, dm, prec, false, 0, nullptr, p, I5, 1.0, &p, I5, g2 / gam, &r, 1.0, nullptr);
            gam = g2;
        }
        if (mixed) fold();
        if (!stagnated || prec == P64 || out.iters >= sp.maxiter) break;
        prec = prec == P16 ? P32 : P64;   // continue one precision up from x_o
        out.inner_used = prec;
    }
    // x_e = D5^-1 (b_e - Dh_eo x_o)
    dense_hop(c, dm, P64, false, 0, &xo, xe, D5Inv(0), -1.0, &be, D5Inv(0), 1.0, nullptr, 0.0, nullptr);
    // true residual of the full system: b_p - D5 x_p - Dh x_pbar
    Half& rt = ws(c, "rt", P64);
    for (int par = 0; par < 2; ++par)
        dense_hop(c, dm, P64, false, par, par ? &xe : &xo, rt, I5, -1.0, par ? &xo : &xe, D5(0), -1.0,
                  par ? &bo : &be, 1.0, c->partial + (size_t)par * nb);
    reduce(c, 2 * nb, S_T0);
    const double rr = read_slot(c, S_T0);
    check_finite(rr, "true residual");
    out.true_resid = std::sqrt(rr) / bnorm;
    out.converged = out.true_resid <= sp.tol;
    return out;
}

int solve_dense_impl(eofa_ctx* c, double m1, double m2, const void* phi, void* chiL, void* chiR, void* Mphi,
                     double* S, const eofa_solver_t* sp, eofa_stats_t* stats) {
    if (!c || !phi || !chiL || !chiR) fail(EOFA_EINVAL, "NULL argument");
    validate_solver(sp);
    if (sp->inner == EOFA_BF16) fail(EOFA_EINVAL, "the dense D_EOFA path has no BF16 inner solver");
    if (!(m1 <= m2)) fail(EOFA_EINVAL, "EOFA needs m1 <= m2");
    double k;
    omega_k(c, m1, m2, &k);
    const auto t0 = std::chrono::steady_clock::now();
    const double f0 = c->flops;
    Half& bLe = ws(c, "bL_e", P64);
    Half& bLo = ws(c, "bL_o", P64);
    Half& bRe = ws(c, "bR_e", P64);
    Half& bRo = ws(c, "bR_o", P64);
    hipchk(launch_eofa_source(phi, c->om, bLe.d, bLo.d, bRe.d, bRo.d, c->L, c->Ls, c->N, c->st), "source");
    Half& ce = ws(c, "chi_e", P64);
    Half& co = ws(c, "chi_o", P64);
    const size_t nmat = (size_t)4 * c->Ls * c->Ls;
    int status = EOFA_OK;
    for (int sys = 0; sys < 2; ++sys) {
        const double mp = m1, mm = sys == 0 ? m1 : m2;
        const std::vector<double> blocks = dense_blocks(c, mp, mm);
        double* dm = (double*)rawbuf(c, sys ? "dense_R" : "dense_L", nmat * sizeof(double));
        hipchk(hipMemcpyAsync(dm, blocks.data(), nmat * sizeof(double), hipMemcpyHostToDevice, c->st),
               "hipMemcpy(dense blocks)");
        hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
        const DenseOut o = solve_dense(c, dm, sys ? bRe : bLe, sys ? bRo : bLo, ce, co, *sp);
        hipchk(launch_dev_to_nat5(sys ? chiR : chiL, ce.d, co.d, c->L, c->Ls, c->N, c->st), "layout");
        if (stats) {
            stats->iters[sys] = o.iters;
            stats->reliable_updates[sys] = o.reliable;
            stats->true_resid[sys] = o.true_resid;
            stats->inner_used[sys] = (eofa_prec_t)o.inner_used;
        }
        if (!o.converged) status = EOFA_ENOCONV;
    }
    if (S || Mphi) {
        const int nb = action_blocks(c->V);
        hipchk(launch_eofa_action(phi, chiL, chiR, c->om, k, Mphi, c->partial, c->V, c->Ls, c->st), "action");
        reduce(c, nb, S_T1);
        const double s = read_slot(c, S_T1);
        check_finite(s, "action");
        if (S) *S = s;
    }
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->flops = c->flops - f0;
    }
    if (status != EOFA_OK) g_err = "solver did not reach the requested true residual";
    return status;
}

void validate_solver(const eofa_solver_t* sp) {
    if (!sp) fail(EOFA_EINVAL, "solver parameters are NULL");
    if (!(sp->tol > 0) || sp->maxiter <= 0) fail(EOFA_EINVAL, "solver tol must be > 0 and maxiter > 0");
    if (sp->inner < EOFA_FP64 || sp->inner > EOFA_BF16) fail(EOFA_EINVAL, "unknown inner precision");
}

void omega_k(const eofa_ctx* c, double m1, double m2, double* k) {
    const double N1 = std::pow(c->b5, c->Ls) + m1 * std::pow(-c->c5, c->Ls);
    const double N2 = std::pow(c->b5, c->Ls) + m2 * std::pow(-c->c5, c->Ls);
    if (!(N1 > 0) || !(N2 > 0)) fail(EOFA_EINVAL, "N(m) = b5^Ls + m (-c5)^Ls must be positive");
    *k = (c->b5 + c->c5) * std::pow(c->b5, 2 * c->Ls - 2) * (m2 - m1) / (N1 * N2);
}

int solve_impl(eofa_ctx* c, double m1, double m2, const void* phi, const void* x0L, const void* x0R,
               void* chiL, void* chiR, void* Mphi, double* S, const eofa_solver_t* sp,
               eofa_stats_t* stats) {
    if (!c || !phi || !chiL || !chiR) fail(EOFA_EINVAL, "NULL argument");
    validate_solver(sp);
    if (!(m1 <= m2)) fail(EOFA_EINVAL, "EOFA needs m1 <= m2");
    double k;
    omega_k(c, m1, m2, &k);
    const auto t0 = std::chrono::steady_clock::now();
    const double f0 = c->flops;
    Half& bLe = ws(c, "bL_e", P64);
    Half& bLo = ws(c, "bL_o", P64);
    Half& bRe = ws(c, "bR_e", P64);
    Half& bRo = ws(c, "bR_o", P64);
    hipchk(launch_eofa_source(phi, c->om, bLe.d, bLo.d, bRe.d, bRo.d, c->L, c->Ls, c->N, c->st), "source");
    Half& ye = ws(c, "y_e", P64);
    Half& yo = ws(c, "y_o", P64);
    Half& ce = ws(c, "chi_e", P64);
    Half& co = ws(c, "chi_o", P64);
    int status = EOFA_OK;
    for (int sys = 0; sys < 2; ++sys) {
        const double mp = m1, mm = sys == 0 ? m1 : m2;
        const void* x0 = sys == 0 ? x0L : x0R;
        if (x0) {   // y0 = Dtilde^-1 chi0
            hipchk(launch_nat5_to_dev(x0, ce.d, co.d, c->L, c->Ls, c->N, c->st), "layout");
            local_op(c, P64, ce, ye, I5, DtInv(c, 0), mp, mm);
            local_op(c, P64, co, yo, I5, DtInv(c, 0), mp, mm);
        }
        // chronological guess from this system's earlier solutions (same masses)
        const int K = x0 ? 0 : c->chrono_k;
        std::vector<Half*> hist, wv;
        int& cnt = c->chrono_n[sys];
        if (K > 0) {
            if (c->chrono_m[sys][0] != mp || c->chrono_m[sys][1] != mm) cnt = 0;
            for (int i = 0; i < K; ++i) {
                hist.push_back(&ws(c, std::string(sys ? "ch_R" : "ch_L") + std::to_string(i), P64));
                wv.push_back(&ws(c, "fc_W" + std::to_string(i), P64));
            }
        }
        const Forecast fc{hist.data(), wv.data(), std::min(cnt, K)};
        CayleyOut o = solve_cayley(c, mp, mm, sys ? bRe : bLe, sys ? bRo : bLo, ye, yo, x0 != nullptr,
                                   ce, co, *sp, K > 0 && cnt > 0 ? &fc : nullptr);
        if (K > 0) {
            convert(c, yo, *hist[cnt % K]);
            ++cnt;
            c->chrono_m[sys][0] = mp;
            c->chrono_m[sys][1] = mm;
        }
        hipchk(launch_dev_to_nat5(sys ? chiR : chiL, ce.d, co.d, c->L, c->Ls, c->N, c->st), "layout");
        if (stats) {
            stats->iters[sys] = o.iters;
            stats->reliable_updates[sys] = o.reliable;
            stats->true_resid[sys] = o.true_resid;
            stats->inner_used[sys] = (eofa_prec_t)o.inner_used;
        }
        if (!o.converged) status = EOFA_ENOCONV;
    }
    if (S || Mphi) {
        const int nb = action_blocks(c->V);
        hipchk(launch_eofa_action(phi, chiL, chiR, c->om, k, Mphi, c->partial, c->V, c->Ls, c->st), "action");
        reduce(c, nb, S_T1);
        const double s = read_slot(c, S_T1);
        check_finite(s, "action");
        if (S) *S = s;
    }
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->flops = c->flops - f0;
    }
    if (status != EOFA_OK) g_err = "solver did not reach the requested true residual";
    return status;
}

// Heatbath of eq. (3.1).  With gamma_l = 1/(1 + beta_l) and h(m) = m / N(m),
//   H(m1) - g Delta_- P_- = H(m+ = m1, m- = mL),  h(mL) = h(m1) + g (h(m2) - h(m1)),
//   H(m2) - g Delta_+ P_+ = H(m+ = mR, m- = m2),  h(mR) = h(m2) + g (h(m1) - h(m2)),
// for g = gamma_l (L side) and g = gamma_l beta_l (R side): every shifted
// operator is an ordinary H(m+, m-), solved in the Cayley form like eofa_solve.
int heatbath_impl(eofa_ctx* c, double m1, double m2, const void* eta, int n, double a0,
                  const double* al, const double* be, int forecast, void* phi, const eofa_solver_t* sp,
                  eofa_stats_t* stats) {
    if (!c || !eta || !phi) fail(EOFA_EINVAL, "NULL argument");
    if (eta == phi) fail(EOFA_EINVAL, "eta and phi may not alias");
    if (n < 0 || n > 64) fail(EOFA_EINVAL, "n_poles must be in [0, 64]");
    if (n > 0 && (!al || !be)) fail(EOFA_EINVAL, "NULL rational coefficients");
    if (forecast < 0 || forecast > 16) fail(EOFA_EINVAL, "forecast must be in [0, 16]");
    validate_solver(sp);
    if (!(m1 <= m2)) fail(EOFA_EINVAL, "EOFA needs m1 <= m2");
    if (!std::isfinite(a0)) fail(EOFA_EINVAL, "alpha0 must be finite");
    double k;
    omega_k(c, m1, m2, &k);
    const double bL = std::pow(c->b5, c->Ls), cL = std::pow(-c->c5, c->Ls);
    auto h = [&](double m) { return m / (bL + m * cL); };
    // h^-1(y) = y b5^Ls / (1 - y (-c5)^Ls); N(h^-1(y)) = b5^Ls / (1 - y (-c5)^Ls) > 0
    auto hinv = [&](double y) {
        const double d = 1.0 - y * cL;
        if (!(d > 0)) fail(EOFA_EINVAL, "a pole shift gives N(m) <= 0");
        return y * bL / d;
    };
    std::vector<double> mL(n), mR(n);
    double c0 = a0;
    for (int l = 0; l < n; ++l) {
        if (!(be[l] > -1.0) || !std::isfinite(be[l]) || !std::isfinite(al[l]))
            fail(EOFA_EINVAL, "rational coefficients must be finite with beta_l > -1");
        const double g = 1.0 / (1.0 + be[l]);
        mL[l] = hinv(h(m1) + g * (h(m2) - h(m1)));
        mR[l] = hinv(h(m2) + g * be[l] * (h(m1) - h(m2)));
        c0 += al[l] * g;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const double f0 = c->flops;
    if (stats) {
        *stats = eofa_stats_t{};
        stats->inner_used[0] = stats->inner_used[1] = sp->inner;
    }
    hipchk(launch_hb_init(eta, phi, c0, (size_t)c->V * 12, c->st), "heatbath");
    int status = EOFA_OK;
    if (k != 0.0 && n > 0) {
        Half& bLe = ws(c, "bL_e", P64);
        Half& bLo = ws(c, "bL_o", P64);
        Half& bRe = ws(c, "bR_e", P64);
        Half& bRo = ws(c, "bR_o", P64);
        hipchk(launch_eofa_source(eta, c->om, bLe.d, bLo.d, bRe.d, bRo.d, c->L, c->Ls, c->N, c->st),
               "source");
        Half& ye = ws(c, "y_e", P64);
        Half& yo = ws(c, "y_o", P64);
        Half& ce = ws(c, "chi_e", P64);
        Half& co = ws(c, "chi_o", P64);
        // per side, a ring of the last `forecast` odd-site solutions (Section 5.2)
        const int K = std::min(forecast, n - 1);
        std::vector<Half*> ring[2], wv;
        for (int i = 0; i < K; ++i) {
            ring[0].push_back(&ws(c, "fc_L" + std::to_string(i), P64));
            ring[1].push_back(&ws(c, "fc_R" + std::to_string(i), P64));
            wv.push_back(&ws(c, "fc_W" + std::to_string(i), P64));
        }
        for (int l = 0; l < n; ++l) {
            const double g = 1.0 / (1.0 + be[l]);
            for (int sys = 0; sys < 2; ++sys) {
                const double mp = sys ? mR[l] : m1, mm = sys ? m2 : mL[l];
                const Forecast fc{ring[sys].data(), wv.data(), std::min(l, K)};
                CayleyOut o = solve_cayley(c, mp, mm, sys ? bRe : bLe, sys ? bRo : bLo, ye, yo, false,
                                           ce, co, *sp, K > 0 ? &fc : nullptr);
                if (K > 0) convert(c, yo, *ring[sys][l % K]);
                // + k g P_- Omega_-^dag y_L,  - k g P_+ Omega_+^dag y_R, weighted by alpha_l g
                const double coef = (sys ? -1.0 : 1.0) * al[l] * g * g * k;
                hipchk(launch_hb_accum(phi, ce.d, co.d, c->om, coef, sys == 0, c->L, c->Ls, c->N, c->st),
                       "heatbath");
                if (stats) {
                    stats->iters[sys] += o.iters;
                    stats->reliable_updates[sys] += o.reliable;
                    stats->true_resid[sys] = std::max(stats->true_resid[sys], o.true_resid);
                    stats->inner_used[sys] = (eofa_prec_t)std::min((int)stats->inner_used[sys], o.inner_used);
                }
                if (!o.converged) status = EOFA_ENOCONV;
            }
        }
    }
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->flops = c->flops - f0;
    }
    if (status != EOFA_OK) g_err = "a heatbath solve did not reach the requested true residual";
    return status;
}

// out = M_EOFA v (eq. (2.5)) for a 4D device field v:
//   M_EOFA v = v - k P_- Omega_-^dag chi_L + k P_+ Omega_+^dag chi_R,
// chi_L = H(m1, m1)^-1 Omega_- P_- v, chi_R = H(m1, m2)^-1 Omega_+ P_+ v (Cayley form).
bool apply_meofa(eofa_ctx* c, double m1, double m2, double k, const void* v, void* out,
                 const eofa_solver_t& sp, eofa_stats_t* stats) {
    Half& bLe = ws(c, "bL_e", P64);
    Half& bLo = ws(c, "bL_o", P64);
    Half& bRe = ws(c, "bR_e", P64);
    Half& bRo = ws(c, "bR_o", P64);
    hipchk(launch_eofa_source(v, c->om, bLe.d, bLo.d, bRe.d, bRo.d, c->L, c->Ls, c->N, c->st), "source");
    hipchk(launch_hb_init(v, out, 1.0, (size_t)c->V * 12, c->st), "meofa");
    Half& ye = ws(c, "y_e", P64);
    Half& yo = ws(c, "y_o", P64);
    Half& ce = ws(c, "chi_e", P64);
    Half& co = ws(c, "chi_o", P64);
    bool ok = true;
    for (int sys = 0; sys < 2; ++sys) {
        CayleyOut o = solve_cayley(c, m1, sys ? m2 : m1, sys ? bRe : bLe, sys ? bRo : bLo, ye, yo, false,
                                   ce, co, sp);
        hipchk(launch_hb_accum(out, ce.d, co.d, c->om, sys ? k : -k, sys == 0, c->L, c->Ls, c->N, c->st),
               "meofa");
        if (stats) {
            stats->iters[sys] += o.iters;
            stats->reliable_updates[sys] += o.reliable;
            stats->true_resid[sys] = std::max(stats->true_resid[sys], o.true_resid);
            stats->inner_used[sys] = (eofa_prec_t)std::min((int)stats->inner_used[sys], o.inner_used);
        }
        ok = ok && o.converged;
    }
    return ok;
}

// Eigenvalues and eigenvectors of a small symmetric matrix A (n x n, row
// major, overwritten) by cyclic Jacobi rotations; Z receives the
// eigenvectors as columns.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double th = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < n; ++r) {   // A <- A J (columns p, q)
                    const double x = A[(size_t)r * n + p], y = A[(size_t)r * n + q];
                    A[(size_t)r * n + p] = cs * x - sn * y;
                    A[(size_t)r * n + q] = sn * x + cs * y;
                }
                for (int r = 0; r < n; ++r) {   // A <- J^T A (rows p, q)
                    const double x = A[(size_t)p * n + r], y = A[(size_t)q * n + r];
                    A[(size_t)p * n + r] = cs * x - sn * y;
                    A[(size_t)q * n + r] = sn * x + cs * y;
                }
                for (int r = 0; r < n; ++r) {   // Z <- Z J
                    const double x = Z[(size_t)r * n + p], y = Z[(size_t)r * n + q];
                    Z[(size_t)r * n + p] = cs * x - sn * y;
                    Z[(size_t)r * n + q] = sn * x + cs * y;
                }
            }
    }
}

// Lanczos on M_EOFA (Hermitian positive definite, Section 2) from `start`:
// the extreme Ritz values of the tridiagonal T_j and their residual norms
// beta_j |s_j| (s_j the last component of the Ritz vector), for choosing the
// interval of the rational heatbath of Section 3.2.
int bounds_impl(eofa_ctx* c, double m1, double m2, const void* start, int n_iter, const eofa_solver_t* sp,
                double* theta, double* resid, eofa_stats_t* stats) {
    if (!c || !start || !theta) fail(EOFA_EINVAL, "NULL argument");
    if (n_iter < 2 || n_iter > 200) fail(EOFA_EINVAL, "n_iter must be in [2, 200]");
    validate_solver(sp);
    if (!(m1 <= m2)) fail(EOFA_EINVAL, "EOFA needs m1 <= m2");
    double k;
    omega_k(c, m1, m2, &k);
    const auto t0 = std::chrono::steady_clock::now();
    const double f0 = c->flops;
    if (stats) {
        *stats = eofa_stats_t{};
        stats->inner_used[0] = stats->inner_used[1] = sp->inner;
    }
    const size_t n = (size_t)c->V * 12;
    const size_t bytes = n * 16;
    void* vb[3] = {rawbuf(c, "lz0", bytes), rawbuf(c, "lz1", bytes), rawbuf(c, "lz2", bytes)};
    const int nb = dot4_blocks(c->V);
    auto dot = [&](const void* a, const void* b) {
        hipchk(launch_dot4(a, b, c->partial, c->V, c->st), "dot");
        reduce(c, nb, S_T0);
        const double r = read_slot(c, S_T0);
        check_finite(r, "Lanczos inner product");
        return r;
    };
    const double s2 = dot(start, start);
    if (!(s2 > 0)) fail(EOFA_EINVAL, "the start vector is zero");
    void* vp = vb[0];
    void* v = vb[1];
    void* w = vb[2];
    hipchk(launch_hb_init(start, v, 1.0 / std::sqrt(s2), n, c->st), "scale");
    std::vector<double> al, be;
    int status = EOFA_OK;
    for (int j = 0; j < n_iter; ++j) {
        if (!apply_meofa(c, m1, m2, k, v, w, *sp, stats)) status = EOFA_ENOCONV;
        const double a = dot(v, w);
        const double b = be.empty() ? 0.0 : be.back();
        hipchk(launch_lanczos_axpy(w, v, be.empty() ? nullptr : vp, a, b, n, c->st), "lanczos");
        al.push_back(a);
        const double bn = std::sqrt(std::max(dot(w, w), 0.0));
        be.push_back(bn);
        if (bn <= 1e-14 * std::fabs(a)) break;   // invariant subspace: T is exact
        hipchk(launch_hb_init(w, vp, 1.0 / bn, n, c->st), "scale");   // v_{j+1} into the old v_{j-1}
        std::swap(vp, v);                                               // vp = v_j, v = v_{j+1}
    }
    const int m = (int)al.size();
    std::vector<double> T((size_t)m * m, 0.0), Z;
    for (int i = 0; i < m; ++i) {
        T[(size_t)i * m + i] = al[i];
        if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = be[i];
    }
    jacobi_eigen(m, T, Z);
    int imin = 0, imax = 0;
    for (int i = 1; i < m; ++i) {
        if (T[(size_t)i * m + i] < T[(size_t)imin * m + imin]) imin = i;
        if (T[(size_t)i * m + i] > T[(size_t)imax * m + imax]) imax = i;
    }
    theta[0] = T[(size_t)imin * m + imin];
    theta[1] = T[(size_t)imax * m + imax];
    if (resid) {
        resid[0] = be[m - 1] * std::fabs(Z[(size_t)(m - 1) * m + imin]);
        resid[1] = be[m - 1] * std::fabs(Z[(size_t)(m - 1) * m + imax]);
    }
    hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->flops = c->flops - f0;
    }
    if (status != EOFA_OK) g_err = "an M_EOFA solve did not reach the requested true residual";
    return status;
}

template <typename F>
int guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const Fail& e) {
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return EOFA_EDEVICE;
    } catch (...) {
        g_err = "unknown error";
        return EOFA_EDEVICE;
    }
}

void free_ctx(eofa_ctx* c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);   // teardown: errors cannot be reported
    for (auto& kv : c->ws) { (void)hipFree(kv.second.d); if (kv.second.nrm) (void)hipFree(kv.second.nrm); }
    for (auto& kv : c->raw) (void)hipFree(kv.second);
    for (int p = 0; p < 4; ++p) if (c->gauge[p]) (void)hipFree(c->gauge[p]);
    for (int p = 0; p < 4; ++p) if (c->sites[p]) (void)hipFree(c->sites[p]);
    if (c->nbr) (void)hipFree(c->nbr);
    for (int p = 0; p < 4; ++p) if (c->nbrb[p]) (void)hipFree(c->nbrb[p]);
    if (c->fsites) (void)hipFree(c->fsites);
    for (int p = 0; p < 4; ++p) if (c->lnkb[p]) (void)hipFree(c->lnkb[p]);
    if (c->U_nat) (void)hipFree(c->U_nat);
    if (c->frag) (void)hipFree(c->frag);
    if (c->frag_b) (void)hipFree(c->frag_b);
    if (c->om) (void)hipFree(c->om);
    if (c->partial) (void)hipFree(c->partial);
    if (c->sc) (void)hipFree(c->sc);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->ring) (void)hipHostFree(c->ring);
    for (auto e : c->ring_ev) if (e) (void)hipEventDestroy(e);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
}

// Cache-blocked traversal of the hopping kernel.  XCD x (of 8) runs one
// contiguous range of logical blocks (see xcd_block), so the site table is
// laid out as 8 regions, one per XCD: the lattice is cut into parts[d]
// pieces along x (in checkerboard positions), y, z and t (their product is
// 8).  Inside a region the sites are visited tile by tile; a tile spans
// `tx`, `ty`, `tz`, `tt` along x, y, z, t (clamped to the region; tx <= 0
// means the region's whole x extent), except along `sweep`, which the tile
// walks one slice at a time.  Every slice then needs the slices before and
// after it along `sweep`, which are still in that XCD's L2, and only the
// tile's faces across the other directions are read again by the
// neighbouring tile.  A checkerboard index does not depend on the parity,
// so the table is the same for both parities.  The sweep may be cut into
// chunks of ext[sweep] slices.  Returns the natural order if the parts do
// not divide the extents.
//
// With `blocks` the same walk runs over the lattice of 2x2x2x2 blocks (parts
// and tile extents count blocks), and every block contributes 8 consecutive
// slots: its sites of either parity, slot j = b_y + 2 b_z + 4 b_t for
// offsets b inside the block (a site's checkerboard index does not depend
// on b_x).  Without a region split that divides the block lattice the blocks
// are listed in natural order.
struct Tiling { int parts[4], sweep, ext[3], tx; };   // dims 0 = x, 1 = y, 2 = z, 3 = t; ext: y, z, t

std::vector<int> site_order(const eofa_ctx* c, const Tiling& T, bool blocks = false) {
    const int Vh = c->Vh, NS = c->NS, nslot = c->nblk_hop * NS;
    std::vector<int> ord;
    ord.reserve(nslot);
    const int hx = c->L[0] / 2;   // checkerboard positions (or blocks) per x row
    const int q = blocks ? 2 : 1;
    const int E[4] = {hx, c->L[1] / q, c->L[2] / q, c->L[3] / q};   // extents in walk units
    // x positions [x0, x1) of the walk row at (y, z, t) in walk units: sites, or blocks of 8 slots
    auto emit = [&](int x0, int x1, int y, int z, int t) {
        if (!blocks) {
            const int cb0 = (c->L[0] * (y + c->L[1] * (z + c->L[2] * t))) / 2;
            for (int i = x0; i < x1; ++i) ord.push_back(cb0 + i);
            return;
        }
        for (int X = x0; X < x1; ++X)
            for (int j = 0; j < 8; ++j) {
                const int yy = 2 * y + (j & 1), zz = 2 * z + ((j >> 1) & 1), tt = 2 * t + (j >> 2);
                ord.push_back(X + hx * (yy + c->L[1] * (zz + c->L[2] * tt)));
            }
    };
    bool ok = T.sweep >= 1 && T.sweep <= 3 && (c->L[0] % 2 == 0) &&
              T.parts[0] * T.parts[1] * T.parts[2] * T.parts[3] == 8;
    for (int d = 0; d < 4 && ok; ++d) ok = T.parts[d] >= 1 && E[d] % T.parts[d] == 0;
    if (blocks && !ok) {
        for (int t = 0; t < E[3]; ++t)
            for (int z = 0; z < E[2]; ++z)
                for (int y = 0; y < E[1]; ++y) emit(0, hx, y, z, t);
    }
    if (ok) {
        int lo[4] = {0, 0, 0, 0}, hi[4] = {E[0], E[1], E[2], E[3]};
        int ext[4] = {T.tx, T.ext[0], T.ext[1], T.ext[2]};
        for (int d = 1; d < 4; ++d) if (ext[d] < 1) ext[d] = 1;
        int od[2], k = 0;   // the two non-sweep dims among y, z, t, slower one first
        for (int d = 3; d >= 1; --d) if (d != T.sweep) od[k++] = d;
        for (int xcd = 0; xcd < 8; ++xcd) {
            int r = xcd;
            for (int d = 0; d < 4; ++d) {   // region of this XCD, x fastest
                const int w = E[d] / T.parts[d], i = r % T.parts[d];
                r /= T.parts[d];
                lo[d] = i * w;
                hi[d] = lo[d] + w;
            }
            const int tx = ext[0] > 0 ? ext[0] : hi[0] - lo[0];
            // the sweep runs in chunks of ext[sweep] slices (all tiles of the
            // region visit one chunk before the next); <= 1 means one chunk
            const int cw = ext[T.sweep] > 1 ? ext[T.sweep] : hi[T.sweep] - lo[T.sweep];
            for (int c0 = lo[T.sweep]; c0 < hi[T.sweep]; c0 += cw)
            for (int a0 = lo[od[0]]; a0 < hi[od[0]]; a0 += ext[od[0]])
                for (int a1 = lo[od[1]]; a1 < hi[od[1]]; a1 += ext[od[1]])
                    for (int x0 = lo[0]; x0 < hi[0]; x0 += tx)
                        for (int v = c0; v < std::min(c0 + cw, hi[T.sweep]); ++v) {
                            int b[4], e[4];
                            b[od[0]] = a0; e[od[0]] = std::min(a0 + ext[od[0]], hi[od[0]]);
                            b[od[1]] = a1; e[od[1]] = std::min(a1 + ext[od[1]], hi[od[1]]);
                            b[T.sweep] = v; e[T.sweep] = v + 1;
                            for (int t = b[3]; t < e[3]; ++t)
                                for (int z = b[2]; z < e[2]; ++z)
                                    for (int y = b[1]; y < e[1]; ++y) emit(x0, std::min(x0 + tx, hi[0]), y, z, t);
                        }
        }
    }
    if ((int)ord.size() != Vh) {
        if (blocks) fail(EOFA_EDEVICE, "internal: block traversal does not cover the lattice");
        ord.resize(Vh);
        for (int i = 0; i < Vh; ++i) ord[i] = i;
    }
    // the table must be a permutation of the sites: check it before use
    std::vector<char> seen(Vh, 0);
    for (int i : ord) {
        if (i < 0 || i >= Vh || seen[i]) fail(EOFA_EDEVICE, "internal: traversal table is not a permutation");
        seen[i] = 1;
    }
    ord.resize(nslot, Vh);   // padding slots are inactive
    return ord;
}

// Block-major neighbour table of a block traversal table `ord`: for output
// parity p, block b of the table (slots 8b..8b+7) and k = 0..4, the
// checkerboard index of slot j's neighbour along its inside direction x
// (k = 0) and its outside direction mu = k - 1, at [p][b][k][j].  The 40
// entries a workgroup's block reads are then 160 contiguous bytes instead of
// 40 scattered rows of the per-direction table.  Padding slots get 0.
std::vector<int> block_neighbours(const eofa_ctx* c, const std::vector<int>& ord) {
    const int nb = (int)ord.size() / 8;
    std::vector<int> out((size_t)2 * nb * 40, 0);
    for (int p = 0; p < 2; ++p)
        for (int b = 0; b < nb; ++b)
            for (int j = 0; j < 8; ++j) {
                const int cb = ord[8 * b + j];
                if (cb >= c->Vh) continue;
                int x[4];
                int r = 2 * cb;
                x[0] = r % c->L[0]; r /= c->L[0];
                x[1] = r % c->L[1]; r /= c->L[1];
                x[2] = r % c->L[2]; x[3] = r / c->L[2];
                x[0] += (p + x[1] + x[2] + x[3]) & 1;
                const int off = (j << 1) | ((__builtin_popcount(j) + p) & 1);
                for (int k = 0; k < 5; ++k) {
                    const int mu = k == 0 ? 0 : k - 1;
                    const bool fwd_inside = ((off >> mu) & 1) == 0;   // +mu lies inside the block
                    const bool fwd = k == 0 ? fwd_inside : !fwd_inside;
                    int e[4] = {x[0], x[1], x[2], x[3]};
                    e[mu] = (e[mu] + (fwd ? 1 : c->L[mu] - 1)) % c->L[mu];
                    const int i = e[0] + c->L[0] * (e[1] + c->L[1] * (e[2] + c->L[2] * e[3]));
                    out[(((size_t)p * nb + b) * 5 + k) * 8 + j] = i >> 1;
                }
            }
    return out;
}

// Default tiling per precision (measured at 24^3x64, Ls = 24, and in a
// model of the per-XCD L2): 8 slabs along z, tiles of 4 (FP16) or 8 (other
// precisions) y rows by the slab's z planes, walked along t.  The block
// traversal of the matrix-core paths (units of 2x2x2x2 blocks): 2 x 4
// regions along y and z, each walked along t one block slice (the region's
// whole x, y, z cross-section) at a time.  Tuning overrides (dims given as y, z or t; in blocks for
// the block traversal):
//   EOFA_TILE="split,ty,tz,tt,sweep"          8 slabs along `split` (e.g. "z,4,3,1,t")
//   EOFA_TILE="p<py>,<pz>,<pt>,ty,tz,tt,sweep" py x pz x pt regions (e.g. "p1,2,4,6,12,1,t")
//   EOFA_TILE="q<px>,<py>,<pz>,<pt>,tx,ty,tz,tt,sweep"  also split and tile x (tx <= 0: whole rows)
//   EOFA_TILE="none"                          natural order
Tiling default_tiling(const eofa_ctx* c, int prec, bool blocks) {
    Tiling T{{1, 1, 1, 1}, 3, {prec == P16 ? 4 : 8, 1, 1}, 0};
    if (blocks) {
        const int by = c->L[1] / 2, bz = c->L[2] / 2, bt = c->L[3] / 2;
        if (by % 2 == 0 && bz % 4 == 0) { T.parts[1] = 2; T.parts[2] = 4; T.ext[0] = by / 2; T.ext[1] = bz / 4; }
        else if (bt % 8 == 0) { T.parts[3] = 8; T.ext[0] = 2; T.ext[1] = bz; }
        else if (bz % 8 == 0) { T.parts[2] = 8; T.ext[0] = 2; T.ext[1] = bz / 8; }
        else T.sweep = 0;   // natural order of the blocks
    } else if (c->L[2] % 8 == 0) { T.parts[2] = 8; T.ext[1] = c->L[2] / 8; }
    else if (c->L[3] % 8 == 0) { T.parts[3] = 8; T.ext[0] = 6; T.ext[1] = 4; }
    else if (c->L[1] % 8 == 0) { T.parts[1] = 8; T.ext[0] = c->L[1] / 8; T.ext[1] = c->L[2]; }
    else T.sweep = 0;   // natural order
    if (const char* e = getenv("EOFA_TILE")) {
        auto dim = [](char ch) { return ch == 'y' ? 1 : ch == 'z' ? 2 : ch == 't' ? 3 : 0; };
        char sp = 0, sw = 0;
        int py = 0, pz = 0, pt = 0, ty = 0, tz = 0, tt = 0;
        int px = 0, tx = 0;
        if (sscanf(e, "q%d,%d,%d,%d,%d,%d,%d,%d,%c", &px, &py, &pz, &pt, &tx, &ty, &tz, &tt, &sw) == 9) {
            T = Tiling{{px, py, pz, pt}, dim(sw), {ty, tz, tt}, tx};
        } else if (sscanf(e, "p%d,%d,%d,%d,%d,%d,%c", &py, &pz, &pt, &ty, &tz, &tt, &sw) == 7) {
            T = Tiling{{1, py, pz, pt}, dim(sw), {ty, tz, tt}, 0};
        } else if (sscanf(e, "%c,%d,%d,%d,%c", &sp, &ty, &tz, &tt, &sw) == 5) {
            T = Tiling{{1, 1, 1, 1}, dim(sw), {ty, tz, tt}, 0};
            if (dim(sp)) T.parts[dim(sp)] = 8;
        } else if (strcmp(e, "none") == 0) {
            T.sweep = 0;
        }
    }
    return T;
}

void load_gauge(eofa_ctx* c, const void* U) {
    const size_t nb = (size_t)4 * c->V * 9 * 16;
    hipchk(hipMemcpyAsync(c->U_nat, U, nb, hipMemcpyDeviceToDevice, c->st), "copy gauge");
    hipchk(launch_ingest_gauge(c->U_nat, c->gauge[P64], c->nbr, c->L, c->Ls, c->aperiodic, c->st), "ingest");
    const size_t nc = (size_t)2 * 8 * 9 * c->Vh;
    for (int p = 1; p < 4; ++p)
        if (c->gauge[p]) hipchk(launch_gauge_convert(p, c->gauge[P64], c->gauge[p], nc, c->st), "gauge convert");
    if (c->frag) hipchk(launch_gauge_c16(c->gauge[P64], c->frag, c->Vh, 0, c->st), "FP16 links");
    if (c->frag_b) hipchk(launch_gauge_c16(c->gauge[P64], c->frag_b, c->Vh, 1, c->st), "BF16 links");
    for (int p : {P64, P32, P16, PB16})
        if (c->lnkb[p]) build_links_blocked(c, p);
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* eofa_last_error(void) { return g_err.c_str(); }

int eofa_ctx_create(eofa_ctx_t** out, const eofa_geom_t* g, const void* U, void* stream) {
    return guarded([&]() -> int {
        if (!out || !g || !U) fail(EOFA_EINVAL, "NULL argument");
        *out = nullptr;
        for (int mu = 0; mu < 4; ++mu)
            if (g->L[mu] < 2 || (g->L[mu] & 1)) fail(EOFA_EINVAL, "every lattice extent must be even and >= 2");
        if (g->Ls < 1 || g->Ls > 64) fail(EOFA_EINVAL, "Ls must be in [1, 64]");
        const double V = (double)g->L[0] * g->L[1] * g->L[2] * g->L[3];
        if (V * g->Ls * 12 > 4.0e9 || V > 1.0e9) fail(EOFA_EINVAL, "lattice too large for 32-bit site indices");
        eofa_ctx* c = new eofa_ctx();
        try {
            hipchk(hipGetDevice(&c->dev), "hipGetDevice");
            init_scratch(c->dev);
            c->st = (hipStream_t)stream;
            for (int mu = 0; mu < 4; ++mu) c->L[mu] = g->L[mu];
            c->Ls = g->Ls;
            c->V = g->L[0] * g->L[1] * g->L[2] * g->L[3];
            c->Vh = c->V / 2;
            c->aperiodic = g->antiperiodic_t ? 1 : 0;
            c->M5 = g->M5;
            c->alpha = g->alpha;
            c->b5 = 0.5 * (g->alpha + 1.0);
            c->c5 = 0.5 * (g->alpha - 1.0);
            c->beta0 = c->b5 * (4.0 - c->M5) + 1.0;
            c->beta1 = c->c5 * (4.0 - c->M5) - 1.0;
            if (c->b5 == 0.0 || c->beta0 == 0.0) fail(EOFA_EINVAL, "degenerate Moebius parameters");
            c->n5 = (size_t)c->Vh * c->Ls;
            c->N = (c->n5 + 255) / 256 * 256;
            // workgroup: NS whole 4D sites x Ls; prefer a multiple of 64 work-items.
            // NS <= 24 keeps the LDS-staged links of the workgroup (FP64:
            // 24 sites x 8 directions x 144 B) within 28 KB.
            int ns = std::min(256 / c->Ls, 24);
            if (ns < 1) ns = 1;
            int best = ns;
            for (int q = ns; q >= 1; --q)
                if ((q * c->Ls) % 64 == 0) { best = q; break; }
            c->NS = best;
            if (const char* e = getenv("EOFA_NS")) {   // tuning override: sites per workgroup
                const int q = atoi(e);
                if (q >= 1 && q <= 24 && q * c->Ls <= 256) c->NS = q;
            }
            c->nblk_hop = (c->Vh + c->NS - 1) / c->NS;
            c->nblk_blas = blas_blocks(c->n5);
            size_t np = (size_t)2 * c->nblk_hop;
            np = std::max(np, (size_t)action_blocks(c->V));
            np = std::max(np, (size_t)md_blocks(4 * c->V));
            np = std::max(np, (size_t)gauge_action_blocks(c->V));
            np = std::max(np, (size_t)2 * c->nblk_blas);   // complex inner products
            c->npartial = np;
            hipchk(hipMalloc((void**)&c->partial, sizeof(double) * np), "hipMalloc(partial)");
            hipchk(hipMalloc((void**)&c->sc, sizeof(double) * S_NSLOT), "hipMalloc(scalars)");
            hipchk(hipMemsetAsync(c->sc, 0, sizeof(double) * S_NSLOT, c->st), "hipMemset");
            hipchk(hipHostMalloc((void**)&c->pinned, sizeof(double) * S_NSLOT, 0), "hipHostMalloc");
            hipchk(hipHostMalloc((void**)&c->ring, sizeof(double) * 8, 0), "hipHostMalloc");
            for (auto& e : c->ring_ev) hipchk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
            hipchk(hipMalloc((void**)&c->nbr, sizeof(int) * 2 * 8 * c->Vh), "hipMalloc(nbr)");
            hipchk(hipMalloc(&c->gauge[P64], (size_t)2 * 8 * 9 * c->Vh * 16), "hipMalloc(gauge)");
            hipchk(hipMalloc(&c->U_nat, (size_t)4 * c->V * 9 * 16), "hipMalloc(U)");
            if (const char* e = getenv("EOFA_NO_MFMA")) c->use_mfma = atoi(e) == 0;
            if (const char* e = getenv("EOFA_MFMA_DEPTH")) c->mfma_depth = atoi(e);
            // block traversal (and block-sharing hops): the FP32 path and the
            // matrix-core paths, whenever a workgroup holds whole 2x2x2x2 blocks
            // and the block form's extra LDS costs no workgroups per CU (at
            // Ls = 8 the links of 24 sites per workgroup already fill it)
            bool blocks_ok = c->NS % 8 == 0;
            int blocks_env = 1;
            if (const char* e = getenv("EOFA_BLOCKS")) blocks_env = atoi(e);   // tuning: 0 off, 2 forced
            blocks_ok = blocks_ok && blocks_env != 0;
            const bool mf_ok = c->use_mfma && c->Ls % 4 == 0;
            for (int p = 0; p < 4; ++p) {
                // (FP64: one link element per staging work-item needs Ls >= 18)
                bool blocks = blocks_ok && (p == P32 || (p == P64 && c->Ls >= 18) ||
                                            (mf_ok && (p == P16 || p == PB16)));
                if (blocks && blocks_env != 2) {
                    const bool mf = p == P16 || p == PB16;
                    const int with = hop_occupancy(p, mf, true, c->NS, c->Ls);
                    blocks = with > 0 && with >= hop_occupancy(p, mf, false, c->NS, c->Ls);
                }
                const std::vector<int> ord = site_order(c, default_tiling(c, p, blocks), blocks);
                c->blk[p] = blocks;
                if (p == P64) {   // the force kernel and the dense hops keep the per-site order (faster for them)
                    const std::vector<int> fo = blocks ? site_order(c, default_tiling(c, P64, false), false) : ord;
                    hipchk(hipMalloc((void**)&c->fsites, sizeof(int) * fo.size()), "hipMalloc(force table)");
                    hipchk(hipMemcpy(c->fsites, fo.data(), sizeof(int) * fo.size(), hipMemcpyHostToDevice),
                           "copy force table");
                }
                if (blocks) {
                    const std::vector<int> nbb = block_neighbours(c, ord);
                    hipchk(hipMalloc((void**)&c->nbrb[p], sizeof(int) * nbb.size()), "hipMalloc(block neighbours)");
                    hipchk(hipMemcpy(c->nbrb[p], nbb.data(), sizeof(int) * nbb.size(), hipMemcpyHostToDevice),
                           "copy block neighbours");
                }
                hipchk(hipMalloc((void**)&c->sites[p], sizeof(int) * ord.size()), "hipMalloc(site table)");
                hipchk(hipMemcpy(c->sites[p], ord.data(), sizeof(int) * ord.size(), hipMemcpyHostToDevice),
                       "copy site table");
            }
            c->om_h.resize(c->Ls);
            for (int s = 0; s < c->Ls; ++s) c->om_h[s] = std::pow(-c->c5 / c->b5, s);
            hipchk(hipMalloc((void**)&c->om, sizeof(double) * c->Ls), "hipMalloc(omega)");
            hipchk(hipMemcpyAsync(c->om, c->om_h.data(), sizeof(double) * c->Ls, hipMemcpyHostToDevice, c->st),
                   "copy omega");
            load_gauge(c, U);
            hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
        } catch (...) {
            free_ctx(c);
            throw;
        }
        *out = c;
        return EOFA_OK;
    });
}

void eofa_ctx_destroy(eofa_ctx_t* c) { free_ctx(c); }

int eofa_ctx_update_gauge(eofa_ctx_t* c, const void* U) {
    return guarded([&]() -> int {
        if (!c || !U) fail(EOFA_EINVAL, "NULL argument");
        load_gauge(c, U);
        return EOFA_OK;
    });
}

int dwf_apply(eofa_ctx_t* c, double mp, double mm, int dagger, int eo, eofa_prec_t prec,
              const void* in, void* out) {
    return guarded([&]() -> int {
        if (!c || !in || !out) fail(EOFA_EINVAL, "NULL argument");
        if (prec < EOFA_FP64 || prec > EOFA_BF16) fail(EOFA_EINVAL, "unknown precision");
        if (eo != 0 && eo != 1) fail(EOFA_EINVAL, "eo must be 0 or 1");
        if (in == out) fail(EOFA_EINVAL, "in and out may not alias");
        const int P = prec;
        Half& ie = ws(c, "ap_in_e", P64);
        Half& io = ws(c, "ap_in_o", P64);
        Half& oe = ws(c, "ap_out_e", P64);
        Half& oo = ws(c, "ap_out_o", P64);
        hipchk(launch_nat5_to_dev(in, ie.d, io.d, c->L, c->Ls, c->N, c->st), "layout");
        Half* pie = &ie; Half* pio = &io; Half* poe = &oe; Half* poo = &oo;
        if (P != P64) {
            pie = &ws(c, "ap_in_e", P); pio = &ws(c, "ap_in_o", P);
            poe = &ws(c, "ap_out_e", P); poo = &ws(c, "ap_out_o", P);
            convert(c, ie, *pie);
            convert(c, io, *pio);
        }
        Half& te = ws(c, "ap_t_e", P);
        Half& to = ws(c, "ap_t_o", P);
        if (eo == 0) {
            for (int par = 0; par < 2; ++par) {
                HopCall h;
                h.prec = P; h.par = par; h.mp = mp; h.mm = mm;
                h.out = par ? poo : poe;
                h.aux = par ? pio : pie;
                h.ca = 1.0; h.ch = 1.0;
                if (!dagger) {
                    // out_p = M_ee in_p + Dh (Dtilde in)_pbar
                    Half& t = par ? te : to;
                    local_op(c, P, par ? *pie : *pio, t, Dt(c, 0), I5, mp, mm);
                    h.in = &t;
                    h.B = Mee(c, 0);
                } else {
                    // out_p = M_ee^dag in_p + Dtilde^dag Dh^dag in_pbar
                    h.dag = true;
                    h.in = par ? pie : pio;
                    h.A = Dt(c, 1);
                    h.B = Mee(c, 1);
                }
                run_hop(c, h);
            }
        } else {
            if (!dagger) {
                local_op(c, P, *pio, to, Dt(c, 0), I5, mp, mm);
                schur_k1(c, P, to, te, mp, mm);
                schur_k2(c, P, te, *pio, *poo, mp, mm, nullptr);
            } else {
                schur_k3(c, P, *pio, te, mp, mm);
                schur_k4(c, P, te, *pio, *poo, mp, mm, nullptr);
            }
            zero(c, *poe);
        }
        if (P != P64) {
            convert(c, *poe, oe);
            convert(c, *poo, oo);
        }
        hipchk(launch_dev_to_nat5(out, oe.d, oo.d, c->L, c->Ls, c->N, c->st), "layout");
        return EOFA_OK;
    });
}

int eofa_solve(eofa_ctx_t* c, double m1, double m2, const void* phi, const void* x0L, const void* x0R,
               void* chiL, void* chiR, void* Mphi, double* S, const eofa_solver_t* sp,
               eofa_stats_t* stats) {
    return guarded([&]() -> int { return solve_impl(c, m1, m2, phi, x0L, x0R, chiL, chiR, Mphi, S, sp, stats); });
}

int eofa_chrono(eofa_ctx_t* c, int depth) {
    return guarded([&] {
        if (!c) fail(EOFA_EINVAL, "NULL argument");
        if (depth < 0 || depth > 16) fail(EOFA_EINVAL, "depth must be in [0, 16]");
        c->chrono_k = depth;
        c->chrono_n[0] = c->chrono_n[1] = 0;
        return EOFA_OK;
    });
}

int eofa_rational_inv_sqrt(double lo, double hi, int n, double* alpha0, double* alpha, double* beta,
                           double* delta_out) {
    return guarded([&] {
        if (!(lo > 0) || !(hi >= lo) || !std::isfinite(hi))
            fail(EOFA_EINVAL, "the interval must satisfy 0 < lo <= hi < inf");
        if (n < 1 || n > 64) fail(EOFA_EINVAL, "n must be in [1, 64]");
        if (!alpha0 || !alpha || !beta) fail(EOFA_EINVAL, "NULL argument");
        zolotarev_inv_sqrt(lo, hi, n, alpha0, alpha, beta, delta_out);
        return EOFA_OK;
    });
}

int eofa_heatbath(eofa_ctx_t* c, double m1, double m2, const void* eta, int n_poles, double alpha0,
                  const double* alpha, const double* beta, int forecast, void* phi, const eofa_solver_t* sp,
                  eofa_stats_t* stats) {
    return guarded([&] {
        return heatbath_impl(c, m1, m2, eta, n_poles, alpha0, alpha, beta, forecast, phi, sp, stats);
    });
}

int eofa_meofa_bounds(eofa_ctx_t* c, double m1, double m2, const void* start, int n_iter,
                      const eofa_solver_t* sp, double* theta_out, double* resid_out, eofa_stats_t* stats) {
    return guarded([&] { return bounds_impl(c, m1, m2, start, n_iter, sp, theta_out, resid_out, stats); });
}

int eofa_force(eofa_ctx_t* c, double m1, double m2, const void* phi, const void* chiL, const void* chiR,
               void* F, void* G, const eofa_solver_t* sp, eofa_stats_t* stats) {
    return guarded([&]() -> int {
        if (!c || !F) fail(EOFA_EINVAL, "NULL argument");
        if (!(m1 <= m2)) fail(EOFA_EINVAL, "EOFA needs m1 <= m2");
        double k;
        omega_k(c, m1, m2, &k);
        int status = EOFA_OK;
        if (!chiL || !chiR) {
            if (!phi) fail(EOFA_EINVAL, "phi is needed when chi is not given");
            const size_t nb5 = (size_t)c->Ls * c->V * 12 * 16;
            void* cl = rawbuf(c, "force_chiL", nb5);
            void* cr = rawbuf(c, "force_chiR", nb5);
            status = solve_impl(c, m1, m2, phi, nullptr, nullptr, cl, cr, nullptr, nullptr, sp, stats);
            if (status != EOFA_OK && status != EOFA_ENOCONV) return status;
            chiL = cl;
            chiR = cr;
        }
        // chi into the FP64 device layout, then one work-item per 5D site
        Half& le = ws(c, "force_chiL_e", P64);
        Half& lo = ws(c, "force_chiL_o", P64);
        Half& re = ws(c, "force_chiR_e", P64);
        Half& ro = ws(c, "force_chiR_o", P64);
        hipchk(launch_nat5_to_dev(chiL, le.d, lo.d, c->L, c->Ls, c->N, c->st), "layout");
        hipchk(launch_nat5_to_dev(chiR, re.d, ro.d, c->L, c->Ls, c->N, c->st), "layout");
        const int ev = timing_begin(c);
        hipchk(launch_force(c->U_nat, le.d, lo.d, re.d, ro.d, c->nbr, c->fsites, k, F, G, c->L, c->Ls,
                            c->aperiodic, c->NS, c->nblk_hop, c->N, c->st), "force");
        // algorithmic bytes: chi_L and chi_R once, U, F (and G)
        timing_end(c, ev, C_FORCE, 2.0 * c->V * c->Ls * 192.0 + 4.0 * c->V * 144.0 * (G ? 3.0 : 2.0));
        hipchk(hipStreamSynchronize(c->st), "hipStreamSynchronize");
        return status;
    });
}

int eofa_md_update(eofa_ctx_t* c, void* U, void* P, const void* F, double dt_p, double dt_u,
                   double* kin) {
    return guarded([&]() -> int {
        if (!c || !U || !P) fail(EOFA_EINVAL, "NULL argument");
        const int nlink = 4 * c->V;
        const int ev = timing_begin(c);
        hipchk(launch_md_update(U, P, F, dt_p, dt_u, nlink, kin ? c->partial : nullptr, c->st), "md update");
        // algorithmic bytes: P (and F) read, P written; U read and written when dt_u != 0
        const bool pf = F && dt_p != 0.0, uu = dt_u != 0.0;
        timing_end(c, ev, C_MD, (double)nlink * 144.0 * ((pf ? 3.0 : 1.0) + (uu ? 2.0 : 0.0)));
        if (kin) {
            reduce(c, md_blocks(nlink), S_T1);
            *kin = read_slot(c, S_T1);
        }
        return EOFA_OK;
    });
}

int eofa_md_update_noalloc(eofa_ctx_t* c, void* U, void* P, const void* F, double dt_p, double dt_u,
                           double* kin_dev) {
    return guarded([&]() -> int {
        if (!c || !U || !P) fail(EOFA_EINVAL, "NULL argument");
        const int nlink = 4 * c->V;
        double* scr = nullptr;
        if (kin_dev) {
            if (md_blocks(nlink) > MD_SCRATCH_DOUBLES)
                fail(EOFA_EINVAL, "lattice too large for eofa_md_update_noalloc: at most " +
                                      std::to_string((long)MD_SCRATCH_DOUBLES * 64) + " sites");
            scr = scratch_of(c->dev);
            if (!scr) fail(EOFA_EDEVICE, "scratch address not initialised for this device");
        }
        // the same kernels as eofa_md_update; every partial the reduction
        // reads is written by this call first, so nothing needs clearing
        hipchk(launch_md_update(U, P, F, dt_p, dt_u, nlink, scr, c->st), "md update");
        if (kin_dev) hipchk(launch_reduce(scr, md_blocks(nlink), kin_dev, 0, c->st), "reduce");
        return EOFA_OK;
    });
}

int eofa_solve_dense(eofa_ctx_t* c, double m1, double m2, const void* phi, void* chiL, void* chiR, void* Mphi,
                     double* S, const eofa_solver_t* sp, eofa_stats_t* stats) {
    return guarded([&]() -> int { return solve_dense_impl(c, m1, m2, phi, chiL, chiR, Mphi, S, sp, stats); });
}

int eofa_gauge_action(eofa_ctx_t* c, const void* U, double beta, double c1, double* S) {
    return guarded([&]() -> int {
        if (!c || !U || !S) fail(EOFA_EINVAL, "NULL argument");
        if (!std::isfinite(beta) || !std::isfinite(c1)) fail(EOFA_EINVAL, "beta and c1 must be finite");
        if (4.0 * c->V > 2147483647.0) fail(EOFA_EINVAL, "lattice too large for 32-bit link indices");
        const int ev = timing_begin(c);
        hipchk(launch_gauge_action(U, c->L, c1, c->partial, c->st), "gauge action");
        // algorithmic bytes: every link read once
        timing_end(c, ev, C_GACTION, 4.0 * c->V * 144.0);
        reduce(c, gauge_action_blocks(c->V), S_T1);
        const double s = read_slot(c, S_T1);
        if (!std::isfinite(s)) fail(EOFA_ENAN, "gauge action is not finite");
        *S = beta * s;
        return EOFA_OK;
    });
}

int eofa_gauge_force(eofa_ctx_t* c, const void* U, double beta, double c1, void* F, int accumulate) {
    return guarded([&]() -> int {
        if (!c || !U || !F) fail(EOFA_EINVAL, "NULL argument");
        if (!std::isfinite(beta) || !std::isfinite(c1)) fail(EOFA_EINVAL, "beta and c1 must be finite");
        if (4.0 * c->V > 2147483647.0) fail(EOFA_EINVAL, "lattice too large for 32-bit link indices");
        if (U == F) fail(EOFA_EINVAL, "F must not alias U");
        const int ev = timing_begin(c);
        hipchk(launch_gauge_force(U, F, c->L, beta, c1, accumulate, c->st), "gauge force");
        // algorithmic bytes: every link read once, F written (and read when accumulating)
        timing_end(c, ev, C_GFORCE, 4.0 * c->V * 144.0 * (accumulate ? 3.0 : 2.0));
        return EOFA_OK;
    });
}

int eofa_timing_enable(eofa_ctx_t* c, int on) {
    return guarded([&]() -> int {
        if (!c) fail(EOFA_EINVAL, "NULL argument");
        timing_collect(c);
        c->timing = on != 0;
        for (int k = 0; k < C_NCLS; ++k) { c->t_count[k] = 0; c->t_ms[k] = 0; c->t_bytes[k] = 0; }
        return EOFA_OK;
    });
}

int eofa_timing_query(eofa_ctx_t* c, const char* name, long* count, double* ms, double* bytes) {
    return guarded([&]() -> int {
        if (!c || !name) fail(EOFA_EINVAL, "NULL argument");
        timing_collect(c);
        long n = 0;
        double t = 0, b = 0;
        bool found = false;
        for (int k = 0; k < C_NCLS; ++k) {
            const bool hit = !strcmp(name, cls_name[k]) || (!strcmp(name, "hop") && k <= C_HOPB16);
            if (hit) { n += c->t_count[k]; t += c->t_ms[k]; b += c->t_bytes[k]; found = true; }
        }
        if (!found) fail(EOFA_EINVAL, std::string("unknown kernel class ") + name);
        if (count) *count = n;
        if (ms) *ms = t;
        if (bytes) *bytes = b;
        return EOFA_OK;
    });
}

}  // extern "C"
