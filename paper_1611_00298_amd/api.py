"""Python binding of the EOFA C ABI: argument marshalling only.

Fields are torch tensors on the GPU, complex128, in the natural layout:
  U   (4, Lt, Lz, Ly, Lx, 3, 3)
  phi (Lt, Lz, Ly, Lx, 4, 3)
  psi (Ls, Lt, Lz, Ly, Lx, 4, 3)
Every computation runs in libeofa.so; torch provides memory and the stream.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import PREC, Geom, Solver, Stats, check

# Iwasaki rectangle coefficient (the gauge action of Table 1); c0 = 1 - 8 c1
IWASAKI_C1 = -0.331


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _want(t, shape, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def make_solver(tol=1e-10, maxiter=20000, inner="fp64", reliable_delta=0.3) -> Solver:
    """inner: "fp64" (plain CGNR), "fp32", "fp16", "bf16", or "fp64_fused"
    (the mixed-precision iteration run in FP64: eofa_solver_t.fused_fp64)."""
    if inner == "fp64_fused":
        return Solver(float(tol), int(maxiter), PREC["fp64"], float(reliable_delta), 1)
    return Solver(float(tol), int(maxiter), PREC[inner], float(reliable_delta), 0)


def rational_inv_sqrt(lo, hi, n):
    """Zolotarev's best relative-error approximation of x^(-1/2) on [lo, hi]:
    x^(-1/2) ~ a0 + sum_l a[l] / (b[l] + x).  Returns (a0, a, b, delta) with
    a, b lists of n floats and delta the maximal relative error."""
    lib = _lib.load()
    n = int(n)
    a = (C.c_double * max(n, 1))()
    b = (C.c_double * max(n, 1))()
    a0 = C.c_double(0.0)
    delta = C.c_double(0.0)
    check(lib.eofa_rational_inv_sqrt(float(lo), float(hi), n, C.byref(a0), a, b, C.byref(delta)))
    return a0.value, list(a)[:n], list(b)[:n], delta.value


class Context:
    """One lattice geometry and gauge field (eofa_ctx_create)."""

    def __init__(self, L, Ls, U, M5=1.8, alpha=2.0, antiperiodic_t=True, stream=None):
        self.lib = _lib.load()
        self.L = tuple(int(v) for v in L)
        self.Ls = int(Ls)
        self.M5 = float(M5)
        self.alpha = float(alpha)
        Lx, Ly, Lz, Lt = self.L
        self.shape4 = (Lt, Lz, Ly, Lx)
        self.shape_gauge = (4,) + self.shape4 + (3, 3)
        self.shape_phi = self.shape4 + (4, 3)
        self.shape5 = (self.Ls,) + self.shape4 + (4, 3)
        _want(U, self.shape_gauge, "U")
        self.device = U.device
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        g = Geom((C.c_int * 4)(*self.L), self.Ls, self.M5, self.alpha, int(bool(antiperiodic_t)))
        h = C.c_void_p()
        check(self.lib.eofa_ctx_create(C.byref(h), C.byref(g), _ptr(U), C.c_void_p(st.cuda_stream)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.eofa_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- eofa_ctx_update_gauge ------------------------------------------------
    def update_gauge(self, U):
        _want(U, self.shape_gauge, "U")
        check(self.lib.eofa_ctx_update_gauge(self.handle, _ptr(U)))

    # -- dwf_apply -------------------------------------------------------------
    def dwf_apply(self, psi, m_plus, m_minus, dagger=False, eo=False, prec="fp64", out=None):
        _want(psi, self.shape5, "psi")
        if out is None:
            out = torch.empty_like(psi)
        _want(out, self.shape5, "out")
        check(self.lib.dwf_apply(self.handle, float(m_plus), float(m_minus), int(bool(dagger)),
                                 int(bool(eo)), PREC[prec], _ptr(psi), _ptr(out)))
        return out

    # -- eofa_solve ------------------------------------------------------------
    def eofa_solve(self, phi, m1, m2, tol=1e-10, maxiter=20000, inner="fp64", reliable_delta=0.3,
                   x0=None, want_mphi=True, allow_noconv=False):
        """Returns (chi_L, chi_R, M_EOFA phi or None, S, stats dict)."""
        _want(phi, self.shape_phi, "phi")
        x0L, x0R = (None, None) if x0 is None else x0
        _want(x0L, self.shape5, "x0_L")
        _want(x0R, self.shape5, "x0_R")
        chiL = torch.empty(self.shape5, dtype=torch.complex128, device=self.device)
        chiR = torch.empty_like(chiL)
        Mphi = torch.empty_like(phi) if want_mphi else None
        S = C.c_double(0.0)
        sp = make_solver(tol, maxiter, inner, reliable_delta)
        st = Stats()
        rc = self.lib.eofa_solve(self.handle, float(m1), float(m2), _ptr(phi), _ptr(x0L), _ptr(x0R),
                                 _ptr(chiL), _ptr(chiR), _ptr(Mphi), C.byref(S), C.byref(sp),
                                 C.byref(st))
        check(rc, allow_noconv)
        d = st.as_dict()
        d["converged"] = rc == _lib.EOFA_OK
        return chiL, chiR, Mphi, S.value, d

    def eofa_solve_dense(self, phi, m1, m2, tol=1e-10, maxiter=20000, inner="fp64", reliable_delta=0.3,
                         want_mphi=True, allow_noconv=False):
        """The same solves on D_EOFA itself, without the Cayley form (the
        comparison path; inner "fp64", "fp32" or "fp16" with reliable updates).
        Returns (chi_L, chi_R, M_EOFA phi or None, S, stats)."""
        _want(phi, self.shape_phi, "phi")
        chiL = torch.empty(self.shape5, dtype=torch.complex128, device=self.device)
        chiR = torch.empty_like(chiL)
        Mphi = torch.empty_like(phi) if want_mphi else None
        S = C.c_double(0.0)
        sp = make_solver(tol, maxiter, inner, reliable_delta)
        st = Stats()
        rc = self.lib.eofa_solve_dense(self.handle, float(m1), float(m2), _ptr(phi), _ptr(chiL), _ptr(chiR),
                                       _ptr(Mphi), C.byref(S), C.byref(sp), C.byref(st))
        check(rc, allow_noconv)
        d = st.as_dict()
        d["converged"] = rc == _lib.EOFA_OK
        return chiL, chiR, Mphi, S.value, d

    # -- eofa_heatbath ---------------------------------------------------------
    def eofa_heatbath(self, eta, m1, m2, coeffs=None, lo=None, hi=None, n_poles=None, tol=1e-10,
                      maxiter=20000, inner="fp64", reliable_delta=0.3, forecast=8, allow_noconv=False):
        """phi ~ M_EOFA^(-1/2) eta (eq. (3.1)).  The rational approximation is
        either coeffs = (a0, a, b) or Zolotarev's on [lo, hi] with n_poles.
        forecast: earlier solutions per side used for chronological initial
        guesses (Section 5.2; 0: start from zero).
        Returns (phi, stats dict); stats carries the approximation error
        "delta" when the coefficients were computed here."""
        _want(eta, self.shape_phi, "eta")
        delta = None
        if coeffs is None:
            if lo is None or hi is None or n_poles is None:
                raise ValueError("give coeffs=(a0, a, b) or lo, hi and n_poles")
            a0, a, b, delta = rational_inv_sqrt(lo, hi, n_poles)
        else:
            a0, a, b = coeffs
        a, b = [float(v) for v in a], [float(v) for v in b]
        if len(a) != len(b):
            raise ValueError("a and b must have the same length")
        n = len(a)
        ca = (C.c_double * max(n, 1))(*a)
        cb = (C.c_double * max(n, 1))(*b)
        phi = torch.empty_like(eta)
        sp = make_solver(tol, maxiter, inner, reliable_delta)
        st = Stats()
        rc = self.lib.eofa_heatbath(self.handle, float(m1), float(m2), _ptr(eta), n, float(a0), ca, cb,
                                    int(forecast), _ptr(phi), C.byref(sp), C.byref(st))
        check(rc, allow_noconv)
        d = st.as_dict()
        d["converged"] = rc == _lib.EOFA_OK
        d["delta"] = delta
        return phi, d

    # -- eofa_chrono ------------------------------------------------------------
    def chrono(self, depth):
        """Chronological initial guesses across solves from the last `depth`
        solutions per system (0: off); clears the history."""
        check(self.lib.eofa_chrono(self.handle, int(depth)))

    # -- eofa_meofa_bounds -----------------------------------------------------
    def meofa_bounds(self, start, m1, m2, n_iter=20, tol=1e-8, maxiter=20000, inner="fp16",
                     reliable_delta=0.3, allow_noconv=False):
        """Extreme eigenvalues of M_EOFA by Lanczos from `start` (4D).
        Returns (theta_min, theta_max, resid_min, resid_max, stats dict)."""
        _want(start, self.shape_phi, "start")
        th = (C.c_double * 2)()
        rs = (C.c_double * 2)()
        sp = make_solver(tol, maxiter, inner, reliable_delta)
        st = Stats()
        rc = self.lib.eofa_meofa_bounds(self.handle, float(m1), float(m2), _ptr(start), int(n_iter),
                                        C.byref(sp), th, rs, C.byref(st))
        check(rc, allow_noconv)
        d = st.as_dict()
        d["converged"] = rc == _lib.EOFA_OK
        return th[0], th[1], rs[0], rs[1], d

    # -- eofa_force ------------------------------------------------------------
    def eofa_force(self, m1, m2, phi=None, chiL=None, chiR=None, want_grad=False, tol=1e-10,
                   maxiter=20000, inner="fp64", reliable_delta=0.3):
        """Returns (F, G or None, stats dict)."""
        _want(phi, self.shape_phi, "phi")
        _want(chiL, self.shape5, "chi_L")
        _want(chiR, self.shape5, "chi_R")
        F = torch.empty(self.shape_gauge, dtype=torch.complex128, device=self.device)
        G = torch.empty_like(F) if want_grad else None
        sp = make_solver(tol, maxiter, inner, reliable_delta)
        st = Stats()
        check(self.lib.eofa_force(self.handle, float(m1), float(m2), _ptr(phi), _ptr(chiL),
                                  _ptr(chiR), _ptr(F), _ptr(G), C.byref(sp), C.byref(st)))
        return F, G, st.as_dict()

    # -- eofa_md_update ----------------------------------------------------------
    def md_update(self, U, P, F=None, dt_p=0.0, dt_u=0.0):
        """In place: P -= dt_p F; U <- exp(i dt_u P) U.  Returns sum tr P^2."""
        _want(U, self.shape_gauge, "U")
        _want(P, self.shape_gauge, "P")
        _want(F, self.shape_gauge, "F")
        kin = C.c_double(0.0)
        check(self.lib.eofa_md_update(self.handle, _ptr(U), _ptr(P), _ptr(F), float(dt_p),
                                      float(dt_u), C.byref(kin)))
        return kin.value

    def md_update_noalloc(self, U, P, F=None, dt_p=0.0, dt_u=0.0, kinetic=None):
        """eofa_md_update_noalloc: the same in-place update, asynchronous and
        allocation-free; with `kinetic` (a float64 CUDA tensor of one
        element) sum tr P^2 is written there on the device."""
        _want(U, self.shape_gauge, "U")
        _want(P, self.shape_gauge, "P")
        _want(F, self.shape_gauge, "F")
        if kinetic is not None:
            if (not isinstance(kinetic, torch.Tensor) or kinetic.device.type != "cuda"
                    or kinetic.dtype != torch.float64 or kinetic.numel() < 1):
                raise TypeError("kinetic must be a float64 CUDA tensor with at least one element")
        check(self.lib.eofa_md_update_noalloc(self.handle, _ptr(U), _ptr(P), _ptr(F), float(dt_p),
                                              float(dt_u), _ptr(kinetic)))
        return kinetic

    # -- gauge action (Table 1: Iwasaki; c1 = 0 is Wilson) -----------------------
    def gauge_action(self, U, beta, c1=IWASAKI_C1):
        """S_g of the field U (any field of this geometry), FP64."""
        _want(U, self.shape_gauge, "U")
        S = C.c_double(0.0)
        check(self.lib.eofa_gauge_action(self.handle, _ptr(U), float(beta), float(c1), C.byref(S)))
        return S.value

    def gauge_force(self, U, beta, c1=IWASAKI_C1, out=None, accumulate=False):
        """F_g = sum_a T^a d^a S_g of U; with accumulate, out += F_g."""
        _want(U, self.shape_gauge, "U")
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs out")
            out = torch.empty_like(U)
        _want(out, self.shape_gauge, "out")
        check(self.lib.eofa_gauge_force(self.handle, _ptr(U), float(beta), float(c1), _ptr(out),
                                        int(bool(accumulate))))
        return out

    # -- timing ------------------------------------------------------------------
    def timing_enable(self, on=True):
        check(self.lib.eofa_timing_enable(self.handle, int(bool(on))))

    def timing_query(self, name="hop"):
        n, ms, b = C.c_long(0), C.c_double(0.0), C.c_double(0.0)
        check(self.lib.eofa_timing_query(self.handle, name.encode(), C.byref(n), C.byref(ms),
                                         C.byref(b)))
        return {"count": n.value, "ms": ms.value, "bytes": b.value}


# Same names as the C entry points, for callers that prefer functions.
def eofa_ctx_create(L, Ls, U, M5=1.8, alpha=2.0, antiperiodic_t=True, stream=None) -> Context:
    return Context(L, Ls, U, M5, alpha, antiperiodic_t, stream)


def eofa_ctx_destroy(ctx: Context):
    ctx.close()


def eofa_ctx_update_gauge(ctx: Context, U):
    ctx.update_gauge(U)


def dwf_apply(ctx: Context, psi, m_plus, m_minus, dagger=False, eo=False, prec="fp64", out=None):
    return ctx.dwf_apply(psi, m_plus, m_minus, dagger, eo, prec, out)


def eofa_solve(ctx: Context, phi, m1, m2, **kw):
    return ctx.eofa_solve(phi, m1, m2, **kw)


def eofa_solve_dense(ctx: Context, phi, m1, m2, **kw):
    return ctx.eofa_solve_dense(phi, m1, m2, **kw)


def eofa_heatbath(ctx: Context, eta, m1, m2, **kw):
    return ctx.eofa_heatbath(eta, m1, m2, **kw)


def eofa_force(ctx: Context, m1, m2, **kw):
    return ctx.eofa_force(m1, m2, **kw)


def eofa_md_update(ctx: Context, U, P, F=None, dt_p=0.0, dt_u=0.0):
    return ctx.md_update(U, P, F, dt_p, dt_u)


def eofa_gauge_action(ctx: Context, U, beta, c1=IWASAKI_C1):
    return ctx.gauge_action(U, beta, c1)


def eofa_gauge_force(ctx: Context, U, beta, c1=IWASAKI_C1, out=None, accumulate=False):
    return ctx.gauge_force(U, beta, c1, out, accumulate)
