"""Plain FP64 CPU oracle for the EOFA hot path (arXiv:1611.00298).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by
the CPU-baseline leg of bench.py, never by the product package.  It shares
no code with the GPU path.

The heavy routines live in ``oracle.c`` (plain C99, OpenMP over sites);
this module loads them with ctypes and exposes numpy-array functions on
fields in the natural layout (see ``dwf_inputs``).  The molecular-dynamics
update and the gauge action (loops as step lists) are written here in numpy.

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_pins.py`` against closed forms, determinant identities,
brute-force dense linear algebra, the free-field dispersion relation, gauge
covariance and finite differences; the gauge action by the closed form of a
uniform abelian flux, gauge invariance and finite differences.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Geom(C.Structure):
    _fields_ = [("L", C.c_int * 4), ("Ls", C.c_int), ("antiperiodic_t", C.c_int),
                ("M5", C.c_double), ("b5", C.c_double), ("c5", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        # OpenMP workers that spin after each parallel region starve the numpy
        # code between oracle calls; let them sleep instead (read at load).
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        _lib = C.CDLL(_LIB)
        P, D, I_, L_ = C.c_void_p, C.c_double, C.c_int, C.c_long
        g = C.POINTER(Geom)
        sigs = {
            "orc_gamma": (None, [I_, P]),
            "orc_wilson": (None, [g, P, P, P, I_, I_]),
            "orc_L": (None, [g, D, D, I_, P, P]),
            "orc_chiral_matrix": (I_, [g, I_, I_, D, P]),
            "orc_apply_chiral": (I_, [g, I_, D, D, I_, P, P]),
            "orc_ddwf": (None, [g, P, D, D, I_, P, P]),
            "orc_deofa": (None, [g, P, D, D, P, P]),
            "orc_g5r5": (None, [g, P, P]),
            "orc_H": (None, [g, P, D, D, P, P]),
            "orc_omega_k": (None, [g, D, D, P, P, P]),
            "orc_schur": (None, [g, P, D, D, I_, P, P]),
            "orc_solve_ddwf_eo": (I_, [g, P, D, D, P, P, D, I_, I_, P]),
            "orc_solve_H": (I_, [g, P, D, D, P, P, D, I_, P]),
            "orc_H_shifted": (None, [g, P, D, D, I_, D, P, P]),
            "orc_solve_H_shifted": (I_, [g, P, D, D, I_, D, P, P, D, I_, P]),
            "orc_eofa_chi": (I_, [g, P, D, D, P, P, P, I_, D, I_, P]),
            "orc_action": (None, [g, D, D, P, P, P, P, P]),
            "orc_force": (None, [g, P, D, D, P, P, P, P, P, L_]),
            "orc_ddwf_sites": (None, [g, P, D, D, I_, P, P, L_, P]),
            "orc_schur_sites": (None, [g, P, D, D, I_, P, P, L_, P]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


class Lattice:
    """Geometry: L = (Lx, Ly, Lz, Lt), Ls, M5 and the Moebius scale alpha.

    b5 = c + d = (alpha + 1)/2 and c5 = c - d = (alpha - 1)/2 with d = 1/2
    (Section 2: c = alpha/2, d = 1/2)."""

    def __init__(self, L, Ls, M5=1.8, alpha=2.0, antiperiodic_t=True):
        self.L = tuple(int(v) for v in L)
        self.Ls = int(Ls)
        self.M5 = float(M5)
        self.alpha = float(alpha)
        self.b5 = (self.alpha + 1.0) / 2.0
        self.c5 = (self.alpha - 1.0) / 2.0
        self.antiperiodic_t = bool(antiperiodic_t)
        self.g = Geom((C.c_int * 4)(*self.L), self.Ls, int(self.antiperiodic_t),
                      self.M5, self.b5, self.c5)
        Lx, Ly, Lz, Lt = self.L
        self.V = Lx * Ly * Lz * Lt
        self.shape4 = (Lt, Lz, Ly, Lx)
        self.shape5 = (self.Ls, Lt, Lz, Ly, Lx, 4, 3)

    @property
    def gp(self):
        return C.byref(self.g)

    def zeros5(self):
        return np.zeros(self.shape5, dtype=np.complex128)

    def parity_mask(self):
        """4D parity p = (x+y+z+t) mod 2 in the natural layout (t,z,y,x)."""
        t, z, y, x = np.indices(self.shape4)
        return (x + y + z + t) % 2


def gamma(mu: int) -> np.ndarray:
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().orc_gamma(mu, _p(out))
    return out


def wilson(lat: Lattice, U, psi, dagger=False):
    """D_w (or D_w^dag) applied slice by slice to a 5D (or 4D) field."""
    psi = _c128(psi)
    nsl = psi.size // (lat.V * 12)
    out = np.empty_like(psi)
    lib().orc_wilson(lat.gp, _p(_c128(U)), _p(psi), _p(out), nsl, int(dagger))
    return out


def L_op(lat: Lattice, mp, mm, psi, transpose=False):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_L(lat.gp, mp, mm, int(transpose), _p(psi), _p(out))
    return out


CHIRAL = {"L": 0, "dtilde": 1, "dtilde_inv": 2, "dperp": 3, "mee": 4, "mee_inv": 5}


def chiral_matrix(lat: Lattice, which: str, plus: bool, m: float) -> np.ndarray:
    A = np.zeros((lat.Ls, lat.Ls))
    rc = lib().orc_chiral_matrix(lat.gp, CHIRAL[which], int(plus), m, _p(A))
    if rc:
        raise ArithmeticError("singular Ls x Ls matrix")
    return A


def apply_chiral(lat: Lattice, which: str, mp, mm, psi, transpose=False):
    psi = _c128(psi)
    out = np.empty_like(psi)
    rc = lib().orc_apply_chiral(lat.gp, CHIRAL[which], mp, mm, int(transpose), _p(psi), _p(out))
    if rc:
        raise ArithmeticError("singular Ls x Ls matrix")
    return out


def ddwf(lat: Lattice, U, mp, mm, psi, dagger=False):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_ddwf(lat.gp, _p(_c128(U)), mp, mm, int(dagger), _p(psi), _p(out))
    return out


def deofa(lat: Lattice, U, mp, mm, psi):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_deofa(lat.gp, _p(_c128(U)), mp, mm, _p(psi), _p(out))
    return out


def g5r5(lat: Lattice, psi):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_g5r5(lat.gp, _p(psi), _p(out))
    return out


def H_op(lat: Lattice, U, mp, mm, psi):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_H(lat.gp, _p(_c128(U)), mp, mm, _p(psi), _p(out))
    return out


def omega_k(lat: Lattice, m1, m2):
    om_m = np.zeros(lat.Ls)
    om_p = np.zeros(lat.Ls)
    k = np.zeros(1)
    lib().orc_omega_k(lat.gp, m1, m2, _p(om_m), _p(om_p), _p(k))
    return om_m, om_p, float(k[0])


def schur(lat: Lattice, U, mp, mm, psi, dagger=False):
    """Mhat (or Mhat^dag) on odd sites of a full-layout 5D field."""
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_schur(lat.gp, _p(_c128(U)), mp, mm, int(dagger), _p(psi), _p(out))
    return out


def solve_ddwf_eo(lat: Lattice, U, mp, mm, b, tol=1e-12, maxiter=10000, fixed=0):
    """Even-odd CGNR solve of D_DWF y = b.  Returns (y, iters, |b - D y|/|b|)."""
    b = _c128(b)
    y = np.zeros_like(b)
    res = np.zeros(1)
    it = lib().orc_solve_ddwf_eo(lat.gp, _p(_c128(U)), mp, mm, _p(b), _p(y), tol, maxiter,
                                 fixed, _p(res))
    return y, it, float(res[0])


def solve_H(lat: Lattice, U, mp, mm, v, tol=1e-12, maxiter=100000):
    v = _c128(v)
    chi = np.zeros_like(v)
    res = np.zeros(1)
    it = lib().orc_solve_H(lat.gp, _p(_c128(U)), mp, mm, _p(v), _p(chi), tol, maxiter, _p(res))
    return chi, it, float(res[0])


def eofa_chi(lat: Lattice, U, m1, m2, phi, method="cayley", tol=1e-12, maxiter=100000):
    """(chi_L, chi_R, iters) of eq. (3.2)'s definitions."""
    chiL = lat.zeros5()
    chiR = lat.zeros5()
    its = np.zeros(2, dtype=np.int32)
    rc = lib().orc_eofa_chi(lat.gp, _p(_c128(U)), m1, m2, _p(_c128(phi)), _p(chiL), _p(chiR),
                            0 if method == "direct" else 1, tol, maxiter, _p(its))
    if rc:
        raise RuntimeError("oracle solve did not converge")
    return chiL, chiR, its


def action(lat: Lattice, m1, m2, phi, chiL, chiR):
    """(S, Im S, M_EOFA phi) of eq. (2.5)."""
    S = np.zeros(2)
    phi = _c128(phi)
    M = np.empty_like(phi)
    lib().orc_action(lat.gp, m1, m2, _p(phi), _p(_c128(chiL)), _p(_c128(chiR)), _p(S), _p(M))
    return float(S[0]), float(S[1]), M


def force(lat: Lattice, U, m1, m2, chiL, chiR, links=None, want_grad=True):
    """Force F = sum_a T^a d^a S of eq. (3.2) and the gradient G.

    links: None (all, arrays shaped like U) or an int array (n, 2) of
    (mu, natural site index) pairs (arrays shaped (n, 3, 3))."""
    U = _c128(U)
    if links is None:
        F = np.zeros_like(U)
        G = np.zeros_like(U) if want_grad else None
        lib().orc_force(lat.gp, _p(U), m1, m2, _p(_c128(chiL)), _p(_c128(chiR)), _p(F), _p(G),
                        None, 0)
    else:
        lk = np.ascontiguousarray(links, dtype=np.int32)
        n = lk.shape[0]
        F = np.zeros((n, 3, 3), dtype=np.complex128)
        G = np.zeros((n, 3, 3), dtype=np.complex128) if want_grad else None
        lib().orc_force(lat.gp, _p(U), m1, m2, _p(_c128(chiL)), _p(_c128(chiR)), _p(F), _p(G),
                        _p(lk), n)
    return F, G


def ddwf_sites(lat: Lattice, U, mp, mm, psi, sites, dagger=False):
    """(D_DWF psi) at sampled (s, natural site) pairs; returns (n, 4, 3)."""
    st = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((st.shape[0], 4, 3), dtype=np.complex128)
    lib().orc_ddwf_sites(lat.gp, _p(_c128(U)), mp, mm, int(dagger), _p(_c128(psi)), _p(st),
                         st.shape[0], _p(out))
    return out


def schur_sites(lat: Lattice, U, mp, mm, psi, sites, dagger=False):
    """(Mhat psi) at sampled (s, odd natural site) pairs; returns (n, 4, 3)."""
    st = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((st.shape[0], 4, 3), dtype=np.complex128)
    lib().orc_schur_sites(lat.gp, _p(_c128(U)), mp, mm, int(dagger), _p(_c128(psi)), _p(st),
                          st.shape[0], _p(out))
    return out


# ---------------------------------------------------------------------------
# molecular dynamics (Section 3: HMC) -- plain numpy
# ---------------------------------------------------------------------------

def expi_hermitian(Q: np.ndarray) -> np.ndarray:
    """exp(i Q) for a stack of Hermitian matrices, by eigen-decomposition."""
    Qh = 0.5 * (Q + np.swapaxes(Q.conj(), -1, -2))
    w, v = np.linalg.eigh(Qh)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def md_update(U, P, F, dt_p, dt_u):
    """P <- P - dt_p F, then U <- exp(i dt_u P) U; returns (U, P)."""
    P = P - dt_p * F
    U = expi_hermitian(dt_u * P) @ U
    return U, P


def kinetic(P) -> float:
    """sum over links of tr(P^2) = (1/2) sum_a (p^a)^2."""
    return float((P * np.swapaxes(P, -1, -2)).sum().real)


# ---------------------------------------------------------------------------
# gauge action of the ensembles (Table 1: Iwasaki) -- plain numpy
#
# S_g = beta sum_x [ c0 sum_{mu<nu} (1 - Re tr W_plaq/3)
#                  + c1 sum_{mu != nu} (1 - Re tr W_rect/3) ],  c0 = 1 - 8 c1,
# W_plaq the 1x1 loop in the (mu, nu) plane and W_rect the loop two links
# long in mu and one in nu.  c1 = -0.331 is the Iwasaki action named in
# Table 1 (the paper gives no coefficients); c1 = 0 is the Wilson action.
# Loops are lists of steps (+-(mu+1)); links are periodic in every direction.
# ---------------------------------------------------------------------------

IWASAKI_C1 = -0.331
_AXIS = (3, 2, 1, 0)   # array axis of direction mu inside U[mu] (t, z, y, x)


def _at(A, d):
    """A(x + d) for an integer 4-vector d (periodic)."""
    return np.roll(A, shift=tuple(-int(v) for v in d), axis=_AXIS)


def _dag(A):
    return np.swapaxes(A.conj(), -1, -2)


def path_product(U, steps, start=(0, 0, 0, 0)):
    """Field of link products along `steps` from x + start, for every x:
    step +(mu+1) multiplies by U_mu(z) and moves z -> z + mu, step -(mu+1)
    moves z -> z - mu and multiplies by U_mu(z)^dag."""
    d = np.array(start, dtype=int)
    M = None
    for st in steps:
        mu = abs(st) - 1
        if st > 0:
            f = _at(U[mu], d)
            d[mu] += 1
        else:
            d[mu] -= 1
            f = _dag(_at(U[mu], d))
        M = f.copy() if M is None else M @ f
    return M


def gauge_loops(c1):
    """(coefficient, steps) of every loop shape in S_g, each summed over x."""
    c0 = 1.0 - 8.0 * c1
    loops = []
    for mu in range(4):
        for nu in range(4):
            a, b = mu + 1, nu + 1
            if mu < nu:
                loops.append((c0, [a, b, -a, -b]))
            if mu != nu and c1 != 0.0:
                loops.append((c1, [a, a, b, -a, -a, -b]))
    return loops


def gauge_action(U, beta, c1=IWASAKI_C1) -> float:
    """S_g by summing every loop over the lattice (definition above)."""
    S = 0.0
    for c, steps in gauge_loops(c1):
        W = path_product(U, steps)
        S += c * float((1.0 - np.trace(W, axis1=-2, axis2=-1).real / 3.0).sum())
    return beta * S


def gauge_staples(U, c1=IWASAKI_C1):
    """Sigma_mu(x) such that S_g depends on U_mu(x) only through
    -(beta/3) Re tr(U_mu(x) Sigma_mu(x)) (plus terms free of U_mu(x)).
    A loop visits U_mu(x) forwards in the rotations of the loop, or of the
    reversed loop (Re tr W = Re tr W^dag), that start with the step +mu; the
    staple is the rest of that rotation, walked from x + mu back to x."""
    out = np.zeros_like(U)
    for c, steps in gauge_loops(c1):
        rev = [-st for st in reversed(steps)]
        for loop in (steps, rev):
            n = len(loop)
            for k in range(n):
                rot = loop[k:] + loop[:k]
                if rot[0] < 0:
                    continue
                mu = rot[0] - 1
                e = [0, 0, 0, 0]
                e[mu] = 1
                out[mu] += c * path_product(U, rot[1:], start=e)
    return out


def gauge_force(U, beta, c1=IWASAKI_C1):
    """F_mu(x) = sum_a T^a d^a S_g, d^a along U_mu(x) -> exp(i eps T^a) U_mu(x),
    T^a = lambda^a/2 (the convention of the fermion force).  With
    Omega = U Sigma: d^a S_g = -(beta/3) Re tr(i T^a Omega), and by the
    completeness of the T^a, F = -(beta/12) (Y - tr(Y)/3), Y = i (Omega - Omega^dag)."""
    Om = U @ gauge_staples(U, c1)
    Y = 1j * (Om - _dag(Om))
    tr = np.trace(Y, axis1=-2, axis2=-1)[..., None, None] / 3.0
    return -(beta / 12.0) * (Y - tr * np.eye(3))


def path_product_at(U, steps, site, start=(0, 0, 0, 0)):
    """path_product at one site (t, z, y, x) only: the same walk, with the
    coordinates wrapped by hand instead of rolled fields."""
    ext = U.shape[1:5]                         # (Lt, Lz, Ly, Lx)
    z = [int(v) for v in site]
    for mu in range(4):
        z[3 - mu] = (z[3 - mu] + start[mu]) % ext[3 - mu]
    M = np.eye(3, dtype=np.complex128)
    for st in steps:
        mu = abs(st) - 1
        if st > 0:
            M = M @ U[(mu,) + tuple(z)]
            z[3 - mu] = (z[3 - mu] + 1) % ext[3 - mu]
        else:
            z[3 - mu] = (z[3 - mu] - 1) % ext[3 - mu]
            M = M @ U[(mu,) + tuple(z)].conj().T
    return M


def gauge_force_at(U, beta, c1, links):
    """gauge_force at the listed links (mu, t, z, y, x) only (for lattices
    too large for the whole-field version); returns (len(links), 3, 3)."""
    out = np.empty((len(links), 3, 3), dtype=np.complex128)
    loops = gauge_loops(c1)
    for n, (mu, *site) in enumerate(links):
        e = [0, 0, 0, 0]
        e[mu] = 1
        sig = np.zeros((3, 3), dtype=np.complex128)
        for c, steps in loops:
            rev = [-st for st in reversed(steps)]
            for loop in (steps, rev):
                for k in range(len(loop)):
                    rot = loop[k:] + loop[:k]
                    if rot[0] == mu + 1:
                        sig += c * path_product_at(U, rot[1:], site, start=e)
        Om = U[(mu,) + tuple(site)] @ sig
        Y = 1j * (Om - Om.conj().T)
        out[n] = -(beta / 12.0) * (Y - np.trace(Y) / 3.0 * np.eye(3))
    return out


# ---------------------------------------------------------------------------
# heatbath (Section 3.2, eq. (3.1)) -- plain numpy on top of H_op
# ---------------------------------------------------------------------------

def zolotarev_inv_sqrt(lo: float, hi: float, n: int):
    """Best relative-error approximation of x^(-1/2) on [lo, hi] by a
    rational function of type (n, n), in the partial-fraction form that
    eq. (3.1) starts from: x^(-1/2) ~ a0 + sum_l a_l / (b_l + x).

    Zolotarev's closed form on y = x/lo in [1, kappa], kappa = hi/lo:
    R0(y) = prod_l (y + c_{2l}) / (y + c_{2l-1}) with
    c_j = sn^2(u_j | m) / cn^2(u_j | m), u_j = j K(m) / (2n + 1),
    m = 1 - 1/kappa (Jacobi elliptic functions of parameter m).
    sqrt(y) R0(y) has its smallest value at y = 1 and its largest at
    y = kappa, and the scale d = 2 / (min + max) makes the relative error
    equioscillate with magnitude delta = (max - min) / (max + min).
    Returns (a0, a, b, delta)."""
    from scipy.special import ellipj, ellipk
    if not (0 < lo <= hi) or n < 1:
        raise ValueError("need 0 < lo <= hi and n >= 1")
    kappa = hi / lo
    m = 1.0 - 1.0 / kappa
    u = np.arange(1, 2 * n + 1) * ellipk(m) / (2 * n + 1)
    sn, cn, _, _ = ellipj(u, m)
    c = (sn / cn) ** 2
    poles, zeros = c[0::2], c[1::2]
    R0 = lambda y: np.prod((y + zeros) / (y + poles))
    fmin, fmax = R0(1.0), np.sqrt(kappa) * R0(kappa)
    d = 2.0 / (fmin + fmax)
    delta = abs(fmax - fmin) / (fmax + fmin)
    # back to x: lo^(-1/2) d prod (x + lo c_2l) / (x + lo c_2l-1), then partial fractions
    A, B = lo * zeros, lo * poles
    a0 = d / np.sqrt(lo)
    a = np.array([a0 * np.prod(A - B[l]) / np.prod(np.delete(B, l) - B[l]) for l in range(n)])
    return float(a0), a, B.copy(), float(delta)


def rational_eval(a0, a, b, x):
    """a0 + sum_l a_l / (b_l + x)."""
    x = np.asarray(x, dtype=np.float64)
    return a0 + sum(al / (bl + x) for al, bl in zip(a, b))


def embed_omega(lat: Lattice, om, v4, lower: bool):
    """The 5D field Omega(s) P v(x): P = P_- (spins 2,3) if lower, else P_+."""
    out = lat.zeros5()
    sl = slice(2, 4) if lower else slice(0, 2)
    out[..., sl, :] = np.asarray(om)[:, None, None, None, None, None, None] * v4[None, ..., sl, :]
    return out


def project_omega(lat: Lattice, om, psi, lower: bool):
    """The 4D field P Omega^dag psi = sum_s Omega(s) P psi(s)."""
    out = np.zeros(lat.shape4 + (4, 3), dtype=np.complex128)
    sl = slice(2, 4) if lower else slice(0, 2)
    out[..., sl, :] = np.einsum("s,s...->...", np.asarray(om), psi[..., sl, :])
    return out


def shifted_H(lat: Lattice, U, m1, m2, which: str, g, psi):
    """The operators inverted in eq. (3.1), with Delta_pm = k Omega_pm Omega_pm^dag:
    'L': [H(m1) - g Delta_- P_-] psi;   'R': [H(m2) - g Delta_+ P_+] psi."""
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_H_shifted(lat.gp, _p(_c128(U)), m1, m2, 0 if which == "L" else 1, g, _p(psi), _p(out))
    return out


def solve_shifted_H(lat: Lattice, U, m1, m2, which: str, g, v, tol=1e-12, maxiter=100000):
    """Solve shifted_H(...) chi = v by CGNR.  Returns (chi, iterations, |v - A chi| / |v|)."""
    v = _c128(v)
    chi = np.zeros_like(v)
    res = np.zeros(1)
    it = lib().orc_solve_H_shifted(lat.gp, _p(_c128(U)), m1, m2, 0 if which == "L" else 1, g,
                                   _p(v), _p(chi), tol, maxiter, _p(res))
    return chi, it, float(res[0])


def eofa_heatbath(lat: Lattice, U, m1, m2, eta, a0, a, b, tol=1e-12, maxiter=100000):
    """phi ~ M_EOFA^(-1/2) eta by eq. (3.1): with gamma_l = 1/(1 + b_l),
    phi = a0 eta + sum_l a_l gamma_l { eta
            + k gamma_l P_- Omega_-^dag [H(m1) - gamma_l Delta_- P_-]^-1 Omega_- P_- eta
            - k gamma_l P_+ Omega_+^dag [H(m2) - gamma_l b_l Delta_+ P_+]^-1 Omega_+ P_+ eta }.
    Two solves per pole.  Returns (phi, iterations per solve)."""
    om_m, om_p, k = omega_k(lat, m1, m2)
    eta = _c128(eta)
    phi = a0 * eta
    vL = embed_omega(lat, om_m, eta, True)
    vR = embed_omega(lat, om_p, eta, False)
    its = []
    for al, bl in zip(a, b):
        g = 1.0 / (1.0 + bl)
        yL, iL, rL = solve_shifted_H(lat, U, m1, m2, "L", g, vL, tol, maxiter)
        yR, iR, rR = solve_shifted_H(lat, U, m1, m2, "R", g * bl, vR, tol, maxiter)
        if rL > tol or rR > tol:
            raise RuntimeError("oracle heatbath solve did not converge")
        its += [iL, iR]
        phi = phi + al * g * (eta + k * g * project_omega(lat, om_m, yL, True)
                              - k * g * project_omega(lat, om_p, yR, False))
    return phi, its
