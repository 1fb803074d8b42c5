"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, a
determinant identity, brute-force dense linear algebra, the free-field
dispersion relation, gauge covariance or finite differences.  Citations
are to arXiv:1611.00298 (sections and equations).
"""
import numpy as np
import pytest
import scipy.linalg

import dwf_inputs as din
import oracle
from helpers import abelian_flux_action, abelian_flux_field
from oracle import Lattice


def dense(fn, shape):
    """Dense matrix of a linear map on complex arrays of the given shape."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = fn(e.reshape(shape)).reshape(n)
    return M


def logdet(M):
    sign, ld = np.linalg.slogdet(M)
    return ld, sign


def rand5(lat, seed):
    return din.gaussian_5d(lat.L, lat.Ls, seed)


TINY = dict(L=(2, 2, 2, 4), Ls=4)


@pytest.fixture(scope="module")
def tiny():
    lat = Lattice(TINY["L"], TINY["Ls"], M5=1.8, alpha=2.0)
    U = din.random_gauge(lat.L, 0.3, 11)
    return lat, U


# --------------------------------------------------------------------------
# conventions: gamma matrices (the paper fixes none; the basis is a reading)
# --------------------------------------------------------------------------

def test_clifford_algebra():
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=1e-15)
    g5 = oracle.gamma(4)
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(g5 @ g[mu], -g[mu] @ g5)


# --------------------------------------------------------------------------
# P1: eq. (2.4), det Dtilde in closed form
# --------------------------------------------------------------------------

@pytest.mark.parametrize("Ls", [2, 3, 4, 8, 24])
@pytest.mark.parametrize("alpha", [1.0, 2.0, 4.0])
def test_dtilde_det_closed_form(Ls, alpha):
    lat = Lattice((2, 2, 2, 2), Ls, alpha=alpha)
    b5, c5 = lat.b5, lat.c5
    for m in (0.0362, 0.3, 1.0):
        for plus in (True, False):
            A = oracle.chiral_matrix(lat, "dtilde", plus, m)
            det = np.linalg.det(A)
            # brute force agrees with b5^Ls + m (-c5)^Ls for every Ls ...
            assert det == pytest.approx(b5 ** Ls + m * (-c5) ** Ls, rel=1e-12)
            # ... and with the paper's (c+d)^Ls + m (c-d)^Ls for even Ls
            if Ls % 2 == 0:
                assert det == pytest.approx(b5 ** Ls + m * c5 ** Ls, rel=1e-12)


def test_dtilde_det_full_lattice(tiny):
    lat, _ = tiny
    m = 0.2
    D = dense(lambda v: oracle.apply_chiral(lat, "dtilde", m, m, v), lat.shape5)
    ld, sign = logdet(D)
    N = lat.b5 ** lat.Ls + m * (-lat.c5) ** lat.Ls
    assert ld == pytest.approx(12 * lat.V * np.log(abs(N)), rel=1e-12)


def test_L_matrix_matches_operator():
    lat = Lattice((2, 2, 2, 2), 5)
    psi = rand5(lat, 3)
    mp, mm = 0.3, 0.7
    ref = np.zeros_like(psi)
    Ap = oracle.chiral_matrix(lat, "L", True, mp)
    Am = oracle.chiral_matrix(lat, "L", False, mm)
    ref[..., :2, :] = np.einsum("st,t...->s...", Ap, psi[..., :2, :])
    ref[..., 2:, :] = np.einsum("st,t...->s...", Am, psi[..., 2:, :])
    assert np.allclose(oracle.L_op(lat, mp, mm, psi), ref, atol=1e-15)
    refT = np.zeros_like(psi)
    refT[..., :2, :] = np.einsum("ts,t...->s...", Ap, psi[..., :2, :])
    refT[..., 2:, :] = np.einsum("ts,t...->s...", Am, psi[..., 2:, :])
    assert np.allclose(oracle.L_op(lat, mp, mm, psi, transpose=True), refT, atol=1e-15)
    # L+^Ls = -m+ (the wrap factor appears once per cycle)
    assert np.allclose(np.linalg.matrix_power(Ap, lat.Ls), -mp * np.eye(lat.Ls))
    assert np.allclose(np.linalg.matrix_power(Am, lat.Ls), -mm * np.eye(lat.Ls))


# --------------------------------------------------------------------------
# P2: eq. (2.3), D_DWF = D_EOFA . Dtilde
# --------------------------------------------------------------------------

def test_ddwf_factorisation_dense(tiny):
    lat, U = tiny
    mp, mm = 0.1, 0.35
    Dd = dense(lambda v: oracle.ddwf(lat, U, mp, mm, v), lat.shape5)
    De = dense(lambda v: oracle.deofa(lat, U, mp, mm, v), lat.shape5)
    Dt = dense(lambda v: oracle.apply_chiral(lat, "dtilde", mp, mm, v), lat.shape5)
    assert np.abs(Dd - De @ Dt).max() < 1e-13
    # the first line of eq. (2.3): (b5 D_w + 1) delta + (c5 D_w - 1) L
    Dw = dense(lambda v: oracle.wilson(lat, U, v), lat.shape5)
    Lm = dense(lambda v: oracle.L_op(lat, mp, mm, v), lat.shape5)
    one = np.eye(Dd.shape[0])
    assert np.abs(Dd - ((lat.b5 * Dw + one) + (lat.c5 * Dw - one) @ Lm)).max() < 1e-13


def test_ddwf_factorisation_matrix_free():
    lat = Lattice((4, 4, 4, 4), 8)
    U = din.random_gauge(lat.L, 0.3, 101)
    psi = rand5(lat, 5)
    a = oracle.ddwf(lat, U, 0.04, 0.04, psi)
    b = oracle.deofa(lat, U, 0.04, 0.04, oracle.apply_chiral(lat, "dtilde", 0.04, 0.04, psi))
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-14


# --------------------------------------------------------------------------
# P3 / P9: Hermiticity of H = g5 R5 D_EOFA (Section 2) and adjoint identities
# --------------------------------------------------------------------------

def test_H_hermitian_dense(tiny):
    lat, U = tiny
    for mp, mm in [(0.1, 0.1), (0.1, 1.0)]:
        H = dense(lambda v: oracle.H_op(lat, U, mp, mm, v), lat.shape5)
        assert np.abs(H - H.conj().T).max() < 1e-14
        # g5 R5 D_DWF is not Hermitian for c5 != 0 (so H is the one to use)
        G = dense(lambda v: oracle.g5r5(lat, oracle.ddwf(lat, U, mp, mm, v)), lat.shape5)
        assert np.abs(G - G.conj().T).max() > 1e-2


def test_wilson_adjoint_dense(tiny):
    lat, U = tiny
    shape4 = lat.shape4 + (4, 3)
    Dw = dense(lambda v: oracle.wilson(lat, U, v), shape4)
    Dwd = dense(lambda v: oracle.wilson(lat, U, v, dagger=True), shape4)
    assert np.abs(Dwd - Dw.conj().T).max() < 1e-15
    g5 = np.kron(np.eye(lat.V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.abs(Dwd - g5 @ Dw @ g5).max() < 1e-15


@pytest.mark.parametrize("name", ["wilson", "L", "ddwf", "schur", "mee_inv", "dtilde"])
def test_adjoint_identity(name):
    lat = Lattice((4, 4, 2, 4), 6)
    U = din.random_gauge(lat.L, 0.4, 7)
    x, y = rand5(lat, 1), rand5(lat, 2)
    mp, mm = 0.05, 0.8
    if name == "schur":
        odd = (lat.parity_mask() == 1)[None, ..., None, None]
        x, y = x * odd, y * odd
    ops = {
        "wilson": lambda v, d: oracle.wilson(lat, U, v, dagger=d),
        "L": lambda v, d: oracle.L_op(lat, mp, mm, v, transpose=d),
        "ddwf": lambda v, d: oracle.ddwf(lat, U, mp, mm, v, dagger=d),
        "schur": lambda v, d: oracle.schur(lat, U, mp, mm, v, dagger=d),
        "mee_inv": lambda v, d: oracle.apply_chiral(lat, "mee_inv", mp, mm, v, transpose=d),
        "dtilde": lambda v, d: oracle.apply_chiral(lat, "dtilde", mp, mm, v, transpose=d),
    }
    op = ops[name]
    lhs = np.vdot(x, op(y, False))
    rhs = np.vdot(op(x, True), y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# --------------------------------------------------------------------------
# P4: Delta_(+/-) = R5 (D_perp(m2) - D_perp(m1)) = k Omega Omega^T (Section 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("Ls", [2, 4, 8, 16, 24])
@pytest.mark.parametrize("alpha", [1.0, 2.0, 4.0])
def test_delta_rank_one(Ls, alpha):
    lat = Lattice((2, 2, 2, 2), Ls, alpha=alpha)
    m1, m2 = 0.0362, 1.0
    om_m, om_p, k = oracle.omega_k(lat, m1, m2)
    R5 = np.eye(Ls)[::-1]
    for plus, om in ((False, om_m), (True, om_p)):
        Dp2 = oracle.chiral_matrix(lat, "dperp", plus, m2)
        Dp1 = oracle.chiral_matrix(lat, "dperp", plus, m1)
        Delta = R5 @ (Dp2 - Dp1)
        assert np.abs(Delta - k * np.outer(om, om)).max() < 1e-13 * max(1, abs(k))
        assert np.linalg.matrix_rank(Delta, tol=1e-10) == 1


def test_shamir_limit():
    """P13: alpha = 1 (Shamir): Omega are unit vectors, k = m2 - m1, Dtilde = 1."""
    lat = Lattice((2, 2, 2, 2), 8, alpha=1.0)
    om_m, om_p, k = oracle.omega_k(lat, 0.04, 1.0)
    assert np.allclose(om_m, np.eye(8)[0])
    assert np.allclose(om_p, np.eye(8)[7])
    assert k == pytest.approx(1.0 - 0.04, rel=1e-14)
    assert np.allclose(oracle.chiral_matrix(lat, "dtilde", True, 0.04), np.eye(8))


# --------------------------------------------------------------------------
# P5 / P6 / P7: eq. (2.1) determinant ratio, HPD, Cayley form, mass split
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def dense_eofa(tiny):
    lat, U = tiny
    m1, m2 = 0.1, 0.6
    H1 = dense(lambda v: oracle.H_op(lat, U, m1, m1, v), lat.shape5)
    H12 = dense(lambda v: oracle.H_op(lat, U, m1, m2, v), lat.shape5)
    H2 = dense(lambda v: oracle.H_op(lat, U, m2, m2, v), lat.shape5)
    return lat, U, m1, m2, H1, H12, H2


def build_M_eofa(lat, U, m1, m2, H1, H12):
    """Dense M_EOFA from the oracle's action routine on unit 4D vectors,
    with chi_L, chi_R from dense solves with H (eq. (3.2) definitions)."""
    shape4 = lat.shape4 + (4, 3)
    n = lat.V * 12
    om_m, om_p, k = oracle.omega_k(lat, m1, m2)
    E = np.eye(n, dtype=np.complex128).reshape((n,) + shape4)
    Pm = E.copy(); Pm[..., :2, :] = 0
    Pp = E.copy(); Pp[..., 2:, :] = 0
    # v(s, x) = Omega(s) P phi(x), one column per unit phi
    vL = np.einsum("s,j...->sj...", om_m, Pm).reshape(lat.Ls, n, -1)
    vR = np.einsum("s,j...->sj...", om_p, Pp).reshape(lat.Ls, n, -1)
    vL = np.moveaxis(vL, 1, -1).reshape(-1, n)
    vR = np.moveaxis(vR, 1, -1).reshape(-1, n)
    XL = np.linalg.solve(H1, vL)
    XR = np.linalg.solve(H12, vR)
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        chiL = XL[:, j].reshape(lat.shape5)
        chiR = XR[:, j].reshape(lat.shape5)
        _, _, Mphi = oracle.action(lat, m1, m2, E[j], chiL, chiR)
        M[:, j] = Mphi.reshape(n)
    return M


def test_eq1_determinant_ratio(dense_eofa):
    lat, U, m1, m2, H1, H12, H2 = dense_eofa
    M = build_M_eofa(lat, U, m1, m2, H1, H12)
    # P6: Hermitian positive definite (Section 2, below eq. (2.1))
    assert np.abs(M - M.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > 0
    # P5: det M_EOFA = det D_EOFA(m2) / det D_EOFA(m1), i.e. eq. (2.1)
    Dd1 = dense(lambda v: oracle.ddwf(lat, U, m1, m1, v), lat.shape5)
    Dd2 = dense(lambda v: oracle.ddwf(lat, U, m2, m2, v), lat.shape5)
    N = lambda m: lat.b5 ** lat.Ls + m * (-lat.c5) ** lat.Ls
    ld_eofa = lambda D, m: logdet(D)[0] - 12 * lat.V * np.log(abs(N(m)))
    lhs = logdet(M)[0]
    rhs = ld_eofa(Dd2, m2) - ld_eofa(Dd1, m1)
    assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-10)
    assert abs(lhs) > 1.0   # the identity is not trivially 0 = 0
    # and the determinant of D_EOFA itself agrees with the factorised form
    De1 = dense(lambda v: oracle.deofa(lat, U, m1, m1, v), lat.shape5)
    assert logdet(De1)[0] == pytest.approx(ld_eofa(Dd1, m1), rel=1e-11)


def test_mass_split_of_R_operator(dense_eofa):
    """P7: H(m2) - Delta_+ P_+ = H(m+ = m1, m- = m2) (eq. (2.5); Section 3.3)."""
    lat, U, m1, m2, H1, H12, H2 = dense_eofa
    R5 = np.eye(lat.Ls)[::-1]
    Dp = R5 @ (oracle.chiral_matrix(lat, "dperp", True, m2)
               - oracle.chiral_matrix(lat, "dperp", True, m1))
    Pp = np.diag([1, 1, 0, 0]).astype(complex)
    DeltaP = np.kron(Dp, np.kron(np.eye(lat.V), np.kron(Pp, np.eye(3))))
    assert np.abs(H2 - DeltaP - H12).max() < 1e-13
    # the opposite assignment differs at O(k)
    H21 = dense(lambda v: oracle.H_op(lat, U, m2, m1, v), lat.shape5)
    assert np.abs(H2 - DeltaP - H21).max() > 1e-2


def test_cayley_form_equals_direct_solve(tiny):
    """P7: H^-1 v = Dtilde D_DWF^-1 g5 R5 v (footnote of Section 5.1)."""
    lat, U = tiny
    phi = din.gaussian_4d(lat.L, 9)
    a = oracle.eofa_chi(lat, U, 0.1, 0.6, phi, method="direct", tol=1e-13)
    b = oracle.eofa_chi(lat, U, 0.1, 0.6, phi, method="cayley", tol=1e-13)
    for x, y in zip(a[:2], b[:2]):
        assert np.linalg.norm(x - y) / np.linalg.norm(x) < 1e-11


def test_equal_masses_trivial(tiny):
    """P14: m1 = m2 gives k = 0, M_EOFA = 1, S = phi^dag phi, F = 0."""
    lat, U = tiny
    phi = din.gaussian_4d(lat.L, 4)
    om_m, om_p, k = oracle.omega_k(lat, 0.3, 0.3)
    assert k == 0.0
    chiL, chiR, _ = oracle.eofa_chi(lat, U, 0.3, 0.3, phi)
    S, Si, M = oracle.action(lat, 0.3, 0.3, phi, chiL, chiR)
    assert S == pytest.approx(np.vdot(phi, phi).real, rel=1e-14)
    assert np.allclose(M, phi)
    F, G = oracle.force(lat, U, 0.3, 0.3, chiL, chiR)
    assert np.abs(F).max() == 0 and np.abs(G).max() == 0


# --------------------------------------------------------------------------
# P10 / P15 / P16: even-odd Schur complement and the CG solvers (Section 5.1)
# --------------------------------------------------------------------------

def test_mee_is_even_even_block(tiny):
    lat, U = tiny
    mp, mm = 0.2, 0.45
    even = (lat.parity_mask() == 0)[None, ..., None, None]
    psi = rand5(lat, 8) * even
    out = oracle.ddwf(lat, U, mp, mm, psi) * even
    ref = oracle.apply_chiral(lat, "mee", mp, mm, psi)
    assert np.abs(out - ref).max() < 1e-14
    # P15: M_ee^-1 M_ee = 1
    for plus, m in ((True, mp), (False, mm)):
        A = oracle.chiral_matrix(lat, "mee", plus, m)
        Ai = oracle.chiral_matrix(lat, "mee_inv", plus, m)
        assert np.abs(Ai @ A - np.eye(lat.Ls)).max() < 1e-14


def test_schur_determinant_identity(tiny):
    """det D = det M_ee * det Mhat (Schur complement) with the oracle's Mhat."""
    lat, U = tiny
    mp, mm = 0.1, 0.3
    D = dense(lambda v: oracle.ddwf(lat, U, mp, mm, v), lat.shape5)
    odd = (lat.parity_mask() == 1)
    odd5 = np.broadcast_to(odd[None, ..., None, None], lat.shape5).reshape(-1)
    idx = np.nonzero(odd5)[0]
    n = lat.V * lat.Ls * 12

    def mhat(vo):
        v = np.zeros(n, dtype=np.complex128)
        v[idx] = vo
        return oracle.schur(lat, U, mp, mm, v.reshape(lat.shape5)).reshape(n)[idx]

    Mh = dense(mhat, (idx.size,))
    ld_mee = sum(6 * (lat.V // 2) * np.log(abs(np.linalg.det(
        oracle.chiral_matrix(lat, "mee", plus, m)))) for plus, m in ((True, mp), (False, mm)))
    assert logdet(D)[0] == pytest.approx(ld_mee + logdet(Mh)[0], rel=1e-12)


def test_eo_solve_matches_dense_solve(tiny):
    lat, U = tiny
    mp, mm = 0.1, 0.6
    b = rand5(lat, 12)
    D = dense(lambda v: oracle.ddwf(lat, U, mp, mm, v), lat.shape5)
    ref = np.linalg.solve(D, b.reshape(-1)).reshape(lat.shape5)
    y, it, res = oracle.solve_ddwf_eo(lat, U, mp, mm, b, tol=1e-13)
    assert res < 1e-12
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-11
    # and the direct H solve agrees with dense linear algebra
    H = dense(lambda v: oracle.H_op(lat, U, mp, mm, v), lat.shape5)
    chi, it, res = oracle.solve_H(lat, U, mp, mm, b, tol=1e-13)
    ref = np.linalg.solve(H, b.reshape(-1)).reshape(lat.shape5)
    assert np.linalg.norm(chi - ref) / np.linalg.norm(ref) < 1e-11


def test_cgnr_fixed_iterations_deterministic(tiny):
    lat, U = tiny
    b = rand5(lat, 13)
    y1, it1, _ = oracle.solve_ddwf_eo(lat, U, 0.1, 0.1, b, fixed=7)
    y2, it2, _ = oracle.solve_ddwf_eo(lat, U, 0.1, 0.1, b, fixed=7)
    assert it1 == it2 == 7
    assert np.array_equal(y1, y2)


# --------------------------------------------------------------------------
# P11: free field, D_w on a plane wave (textbook closed form)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 8, 6)])
def test_free_field_plane_wave(L):
    lat = Lattice(L, 1, M5=1.8)
    U = np.zeros((4,) + lat.shape4 + (3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    g = np.random.default_rng(1)
    Lx, Ly, Lz, Lt = L
    n = [1, 2, 3]
    p = np.array([2 * np.pi * n[0] / Lx, 2 * np.pi * n[1] / Ly, 2 * np.pi * n[2] / Lz,
                  (2 * 1 + 1) * np.pi / Lt])   # antiperiodic in t
    t, z, y, x = np.indices(lat.shape4)
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
    psi = ph[..., None, None] * u
    out = oracle.wilson(lat, U, psi[None])[0]
    gam = [oracle.gamma(mu) for mu in range(4)]
    Mp = (4 - 1.8 - np.cos(p).sum()) * np.eye(4) + 1j * sum(gam[mu] * np.sin(p[mu]) for mu in range(4))
    ref = ph[..., None, None] * (Mp @ u)
    assert np.abs(out - ref).max() < 1e-13


# --------------------------------------------------------------------------
# P12: gauge covariance of D_w and of the action
# --------------------------------------------------------------------------

def gauge_transform(lat, U, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag."""
    ax = {0: 3, 1: 2, 2: 1, 3: 0}
    Ug = np.empty_like(U)
    for mu in range(4):
        gxmu = np.roll(g, -1, axis=ax[mu])
        Ug[mu] = g @ U[mu] @ np.swapaxes(gxmu.conj(), -1, -2)
    return Ug


def test_gauge_covariance():
    lat = Lattice((4, 2, 4, 4), 4)
    U = din.random_gauge(lat.L, 0.5, 21)
    g = din.random_su3(lat.shape4, 1.0, 22)
    Ug = gauge_transform(lat, U, g)
    psi = rand5(lat, 23)
    gpsi = np.einsum("tzyxab,stzyxcb->stzyxca", g, psi)
    a = oracle.wilson(lat, Ug, gpsi)
    b = np.einsum("tzyxab,stzyxcb->stzyxca", g, oracle.wilson(lat, U, psi))
    assert np.abs(a - b).max() < 1e-13
    phi = din.gaussian_4d(lat.L, 24)
    gphi = np.einsum("tzyxab,tzyxcb->tzyxca", g, phi)
    m1, m2 = 0.05, 0.5
    S0 = oracle.action(lat, m1, m2, phi, *oracle.eofa_chi(lat, U, m1, m2, phi, tol=1e-13)[:2])[0]
    S1 = oracle.action(lat, m1, m2, gphi, *oracle.eofa_chi(lat, Ug, m1, m2, gphi, tol=1e-13)[:2])[0]
    assert S1 == pytest.approx(S0, rel=1e-11)


# --------------------------------------------------------------------------
# P8: eq. (3.2) force against central finite differences
# --------------------------------------------------------------------------

def test_force_finite_difference():
    lat = Lattice((2, 2, 4, 4), 4)
    U = din.random_gauge(lat.L, 0.4, 31)
    phi = din.gaussian_4d(lat.L, 32)
    m1, m2 = 0.05, 0.7

    def S_of(Ux):
        chiL, chiR, _ = oracle.eofa_chi(lat, Ux, m1, m2, phi, tol=1e-14)
        return oracle.action(lat, m1, m2, phi, chiL, chiR)[0]

    chiL, chiR, _ = oracle.eofa_chi(lat, U, m1, m2, phi, tol=1e-14)
    F, G = oracle.force(lat, U, m1, m2, chiL, chiR)
    assert np.abs(F - np.swapaxes(F.conj(), -1, -2)).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14
    T = din.gell_mann() / 2
    rng = np.random.default_rng(5)
    d = 1e-5
    for _ in range(4):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in lat.shape4)
        a = int(rng.integers(8))
        Up, Um = U.copy(), U.copy()
        Up[(mu,) + site] = scipy.linalg.expm(1j * d * T[a]) @ U[(mu,) + site]
        Um[(mu,) + site] = scipy.linalg.expm(-1j * d * T[a]) @ U[(mu,) + site]
        fd = (S_of(Up) - S_of(Um)) / (2 * d)
        an = 2 * np.trace(T[a] @ F[(mu,) + site]).real   # F = sum_a T^a d^a S
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-8)
        # complex direction for the matrix gradient: dS = Re tr(G^dag dU)
        E = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Up, Um = U.copy(), U.copy()
        Up[(mu,) + site] += d * E
        Um[(mu,) + site] -= d * E
        fd = (S_of(Up) - S_of(Um)) / (2 * d)
        an = np.trace(G[(mu,) + site].conj().T @ E).real
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-8)


# --------------------------------------------------------------------------
# sampled single-site evaluation agrees with the full-field operators
# --------------------------------------------------------------------------

def test_sampled_operators():
    lat = Lattice((4, 4, 2, 4), 6)
    U = din.random_gauge(lat.L, 0.4, 41)
    psi = rand5(lat, 42)
    mp, mm = 0.04, 0.9
    rng = np.random.default_rng(3)
    par = lat.parity_mask().reshape(-1)
    odd_sites = np.nonzero(par == 1)[0]
    sites = np.stack([rng.integers(lat.Ls, size=20), rng.choice(odd_sites, size=20)], 1)
    for dag in (False, True):
        full = oracle.ddwf(lat, U, mp, mm, psi, dagger=dag).reshape(lat.Ls, lat.V, 4, 3)
        smp = oracle.ddwf_sites(lat, U, mp, mm, psi, sites, dagger=dag)
        assert np.abs(smp - full[sites[:, 0], sites[:, 1]]).max() < 1e-13
        full = oracle.schur(lat, U, mp, mm, psi, dagger=dag).reshape(lat.Ls, lat.V, 4, 3)
        smp = oracle.schur_sites(lat, U, mp, mm, psi, sites, dagger=dag)
        assert np.abs(smp - full[sites[:, 0], sites[:, 1]]).max() < 1e-13


# --------------------------------------------------------------------------
# molecular dynamics helpers (Section 3)
# --------------------------------------------------------------------------

def test_md_exponential():
    P = din.gaussian_momenta((2, 2, 2, 2), 7)
    Q = 0.1 * P
    E = oracle.expi_hermitian(Q)
    flat_Q = Q.reshape(-1, 3, 3)[:16]
    for q, e in zip(flat_Q, E.reshape(-1, 3, 3)[:16]):
        assert np.abs(e - scipy.linalg.expm(1j * q)).max() < 1e-14
    EE = E @ np.swapaxes(E.conj(), -1, -2)
    assert np.abs(EE - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(E) - 1).max() < 1e-14
    # kinetic term: tr P^2 = (1/2) sum_a (p^a)^2
    p = din.rng(7).standard_normal((4, 2, 2, 2, 2, 8))
    assert oracle.kinetic(P) == pytest.approx(0.5 * (p ** 2).sum(), rel=1e-12)


def _md_hamiltonian(U, P, beta, c1):
    return oracle.kinetic(P) + oracle.gauge_action(U, beta, c1)


def _leapfrog(U, P, beta, c1, n, dt, update):
    """n leapfrog steps of length dt, each call of `update` kicking P with
    the force at the current links and then drifting U with the new P."""
    U, P = update(U, P, oracle.gauge_force(U, beta, c1), 0.5 * dt, dt)
    for _ in range(1, n):
        U, P = update(U, P, oracle.gauge_force(U, beta, c1), dt, dt)
    return update(U, P, oracle.gauge_force(U, beta, c1), 0.5 * dt, 0.0)


def _md_pin(update):
    """Energy error at three step sizes over a fixed trajectory length, and
    the distance of a forward-then-reversed trajectory from its start."""
    L, beta, c1, tau = (4, 4, 4, 4), 5.7, 0.0, 0.5
    U0 = din.random_gauge(L, 0.5, 131)
    P0 = din.gaussian_momenta(L, 132)
    H0 = _md_hamiltonian(U0, P0, beta, c1)
    dH = []
    for n in (4, 8, 16):
        U, P = _leapfrog(U0, P0, beta, c1, n, tau / n, update)
        dH.append(_md_hamiltonian(U, P, beta, c1) - H0)
        if n == 8:
            Ur, Pr = _leapfrog(U, -P, beta, c1, n, tau / n, update)
            rev = max(np.abs(Ur - U0).max(), np.abs(Pr + P0).max())
    return dH, rev


def test_md_update_leapfrog():
    """HMC molecular dynamics (Section 3) with the oracle's update and its
    finite-difference-pinned gauge force: the equations of motion
    dU/dt = iPU, dP/dt = -F conserve H = tr P^2 + S_g, so leapfrog's energy
    error falls as dt^2 (a factor of 4 per halving), and the integrator is
    reversible: flipping P and integrating again returns to (U0, -P0)."""
    dH, rev = _md_pin(oracle.md_update)
    for a, b in zip(dH, dH[1:]):
        assert 3.0 < a / b < 5.0, dH
    assert rev < 1e-12


def test_md_update_pin_detects_planted_mistakes():
    """The leapfrog pin above fails for the two plausible slips in the
    update: the wrong sign of the force kick (P + dt F) and a drift that
    uses the momenta from before the kick."""
    def wrong_sign(U, P, F, dt_p, dt_u):
        P = P + dt_p * F
        return oracle.expi_hermitian(dt_u * P) @ U, P

    def stale_momenta(U, P, F, dt_p, dt_u):
        return oracle.expi_hermitian(dt_u * P) @ U, P - dt_p * F

    for update in (wrong_sign, stale_momenta):
        dH, rev = _md_pin(update)
        scales = all(3.0 < a / b < 5.0 for a, b in zip(dH, dH[1:]))
        assert not (scales and rev < 1e-12), update.__name__


# --------------------------------------------------------------------------
# heatbath (Section 3.2, eq. (3.1))
# --------------------------------------------------------------------------

def alternation_runs(e, level):
    """Number of same-sign runs among the samples where |e| reaches level."""
    s = np.sign(e[np.abs(e) >= level])
    return 1 + int(np.sum(s[1:] != s[:-1]))


@pytest.mark.parametrize("lo,hi,n", [(0.5, 5.0, 3), (0.9, 2.7, 4), (1.0, 100.0, 6), (0.2, 0.3, 2),
                                     (0.05, 50.0, 10)])
def test_zolotarev_equioscillation(lo, hi, n):
    """Chebyshev's alternation theorem: a type (n, n) rational function whose
    relative error against x^(-1/2) takes its extreme value with alternating
    signs at 2n + 2 points is the best one, so the returned coefficients are
    the minimax approximation and delta is its error."""
    a0, a, b, delta = oracle.zolotarev_inv_sqrt(lo, hi, n)
    x = np.exp(np.linspace(np.log(lo), np.log(hi), 400001))
    e = np.sqrt(x) * oracle.rational_eval(a0, a, b, x) - 1.0
    assert np.abs(e).max() == pytest.approx(delta, rel=1e-6)
    assert alternation_runs(e, 0.98 * delta) == 2 * n + 2
    assert np.all(b > 0)    # gamma_l = 1 / (1 + b_l) lies in (0, 1)
    # one pole fewer is strictly worse
    if n > 1:
        assert oracle.zolotarev_inv_sqrt(lo, hi, n - 1)[3] > 2 * delta


def test_zolotarev_degenerate_interval():
    """lo = hi: x^(-1/2) is matched exactly at the single point."""
    a0, a, b, delta = oracle.zolotarev_inv_sqrt(2.0, 2.0, 2)
    assert delta == 0.0
    assert oracle.rational_eval(a0, a, b, 2.0) == pytest.approx(2.0 ** -0.5, rel=1e-14)


@pytest.mark.parametrize("alpha,Ls", [(1.0, 4), (2.0, 5), (4.0, 6)])
def test_shifted_operators_are_mass_shifts(alpha, Ls):
    """The operators of eq. (3.1) are again H(m+, m-) with one boundary mass
    moved: with h(m) = m / N(m), N(m) = b5^Ls + m (-c5)^Ls,
    H(m1) - g Delta_- P_- = H(m+ = m1, m- = mL), h(mL) = h(m1) + g (h(m2) - h(m1)),
    H(m2) - g Delta_+ P_+ = H(m+ = mR, m- = m2), h(mR) = h(m2) + g (h(m1) - h(m2))."""
    lat = Lattice((4, 2, 2, 4), Ls, M5=1.8, alpha=alpha)
    U = din.random_gauge(lat.L, 0.3, 12)
    psi = rand5(lat, 13)
    m1, m2 = 0.04, 0.7
    N = lambda m: lat.b5 ** Ls + m * (-lat.c5) ** Ls
    h = lambda m: m / N(m)
    hinv = lambda y: y * lat.b5 ** Ls / (1.0 - y * (-lat.c5) ** Ls)
    for g in (0.0, 0.3, 0.8, 1.0):
        mL = hinv(h(m1) + g * (h(m2) - h(m1)))
        mR = hinv(h(m2) + g * (h(m1) - h(m2)))
        A = oracle.shifted_H(lat, U, m1, m2, "L", g, psi)
        B = oracle.shifted_H(lat, U, m1, m2, "R", g, psi)
        scale = np.abs(A).max()
        assert np.abs(A - oracle.H_op(lat, U, m1, mL, psi)).max() < 1e-14 * scale
        assert np.abs(B - oracle.H_op(lat, U, mR, m2, psi)).max() < 1e-14 * scale
        if 0 < g:   # the other chirality's mass is not the one that moves
            assert np.abs(A - oracle.H_op(lat, U, mL, m1, psi)).max() > 1e-3 * scale


@pytest.fixture(scope="module")
def dense_heatbath(dense_eofa):
    lat, U, m1, m2, H1, H12, H2 = dense_eofa
    M = build_M_eofa(lat, U, m1, m2, H1, H12)
    M = 0.5 * (M + M.conj().T)
    lam, V = np.linalg.eigh(M)
    eta = din.gaussian_4d(lat.L, 31)
    return lat, U, m1, m2, M, lam, V, eta


def test_heatbath_is_the_rational_function_of_M(dense_heatbath):
    """eq. (3.1) (2 N_p solves with H) equals a0 eta + sum_l a_l (b_l + M)^-1 eta
    with M = M_EOFA built densely: checks the Sherman-Morrison form, the
    gamma_l b_l weight of the R-side shift and the signs."""
    lat, U, m1, m2, M, lam, V, eta = dense_heatbath
    a0, a, b, delta = oracle.zolotarev_inv_sqrt(0.9 * lam[0], 1.1 * lam[-1], 3)
    phi, its = oracle.eofa_heatbath(lat, U, m1, m2, eta, a0, a, b, tol=1e-13)
    n = M.shape[0]
    e = eta.reshape(n)
    ref = a0 * e + sum(al * np.linalg.solve(M + bl * np.eye(n), e) for al, bl in zip(a, b))
    assert np.linalg.norm(phi.reshape(n) - ref) / np.linalg.norm(ref) < 1e-11
    assert len(its) == 6 and min(its) > 0


def test_heatbath_draws_from_M_eofa(dense_heatbath):
    """phi = M^(-1/2) eta to within the approximation's error: with the
    spectrum inside [lo, hi], |phi - M^(-1/2) eta| <= delta |M^(-1/2) eta|,
    and phi^dag M phi = eta^dag eta (1 + O(delta)) (Section 3.2)."""
    lat, U, m1, m2, M, lam, V, eta = dense_heatbath
    assert lam[0] > 0 and lam[-1] / lam[0] > 1.05    # a non-trivial spectrum
    n = M.shape[0]
    e = eta.reshape(n)
    exact = V @ ((V.conj().T @ e) / np.sqrt(lam))
    for npole in (2, 5):
        a0, a, b, delta = oracle.zolotarev_inv_sqrt(lam[0], lam[-1], npole)
        phi, _ = oracle.eofa_heatbath(lat, U, m1, m2, eta, a0, a, b, tol=1e-13)
        p = phi.reshape(n)
        err = np.linalg.norm(p - exact) / np.linalg.norm(exact)
        assert err <= delta * (1 + 1e-6) + 1e-11
        if npole == 2:
            assert err > 1e-3 * delta     # the bound is not vacuous here
        S = np.vdot(p, M @ p).real
        assert abs(S / np.vdot(e, e).real - 1) <= 2.01 * delta + 1e-11


# --------------------------------------------------------------------------
# P12: gauge action of the ensembles (Table 1: Iwasaki; c1 = 0 is Wilson)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("c1", [0.0, oracle.IWASAKI_C1])
def test_gauge_unit_field(c1):
    lat = Lattice((4, 4, 4, 6), 1)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4,) + lat.shape4 + (3, 3)).copy()
    assert oracle.gauge_action(U, 2.13, c1) == 0.0
    assert np.abs(oracle.gauge_force(U, 2.13, c1)).max() == 0.0


@pytest.mark.parametrize("c1", [0.0, oracle.IWASAKI_C1, 0.25])
def test_gauge_abelian_flux_closed_form(c1):
    """Closed form of the action (each plane a different flux, so a dropped
    plane, orientation or rectangle term shows), checked after a random gauge
    rotation; the uniform flux is a stationary point, so the force vanishes."""
    L = (4, 6, 4, 8)
    quanta = {(0, 1): 1, (0, 2): 2, (0, 3): 3, (1, 2): 1, (1, 3): 5, (2, 3): 2}
    U, F = abelian_flux_field(L, quanta)
    beta = 1.7
    S_ref = abelian_flux_action(L, F, beta, c1)
    lat = Lattice(L, 1)
    g = din.random_su3(lat.shape4, 1.0, 121)
    Ug = gauge_transform(lat, U, g)
    for V in (U, Ug):
        assert oracle.gauge_action(V, beta, c1) == pytest.approx(S_ref, rel=1e-12)
        assert np.abs(oracle.gauge_force(V, beta, c1)).max() < 1e-12 * beta * lat.V
    # a non-uniform field is not stationary: the vanishing above is not trivial
    U2 = U.copy()
    U2[1, 0, 0, 0, 0] = din.random_su3((), 0.5, 122) @ U2[1, 0, 0, 0, 0]
    assert np.abs(oracle.gauge_force(U2, beta, c1)).max() > 1e-2


@pytest.mark.parametrize("c1", [0.0, oracle.IWASAKI_C1])
def test_gauge_invariance_and_covariance(c1):
    lat = Lattice((4, 2, 4, 6), 1)
    U = din.random_gauge(lat.L, 0.6, 123)
    g = din.random_su3(lat.shape4, 1.0, 124)
    Ug = gauge_transform(lat, U, g)
    assert oracle.gauge_action(Ug, 2.0, c1) == pytest.approx(oracle.gauge_action(U, 2.0, c1), rel=1e-13)
    F, Fg = oracle.gauge_force(U, 2.0, c1), oracle.gauge_force(Ug, 2.0, c1)
    assert np.abs(Fg - g @ F @ np.swapaxes(g.conj(), -1, -2)).max() < 1e-12
    # traceless Hermitian
    assert np.abs(F - np.swapaxes(F.conj(), -1, -2)).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13


@pytest.mark.parametrize("c1", [0.0, oracle.IWASAKI_C1])
def test_gauge_force_finite_difference(c1):
    """d^a S_g = 2 tr(T^a F) against Richardson-extrapolated central
    differences along U_mu(x) -> exp(i eps T^a) U_mu(x)."""
    lat = Lattice((4, 4, 2, 6), 1)
    U = din.random_gauge(lat.L, 0.7, 125)
    beta = 2.25
    F = oracle.gauge_force(U, beta, c1)
    T = din.gell_mann() / 2
    r = np.random.default_rng(126)
    for _ in range(6):
        mu = int(r.integers(4))
        site = tuple(int(r.integers(n)) for n in lat.shape4)
        a = int(r.integers(8))

        def S_at(e):
            V = U.copy()
            V[(mu,) + site] = oracle.expi_hermitian(e * T[a]) @ V[(mu,) + site]
            return oracle.gauge_action(V, beta, c1)

        h = 1e-3
        d1 = (S_at(h) - S_at(-h)) / (2 * h)
        d2 = (S_at(h / 2) - S_at(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
        an = 2 * np.trace(T[a] @ F[(mu,) + site]).real
        assert an == pytest.approx(fd, rel=1e-7, abs=1e-8)


def test_gauge_force_pointwise_matches_field():
    """The pointwise walk (used at full lattice size) equals the pinned
    whole-field force, including links on the wrapped boundary."""
    lat = Lattice((4, 2, 6, 4), 1)
    U = din.random_gauge(lat.L, 0.7, 127)
    F = oracle.gauge_force(U, 1.9, oracle.IWASAKI_C1)
    r = np.random.default_rng(128)
    links = [(int(r.integers(4)),) + tuple(int(r.integers(n)) for n in lat.shape4) for _ in range(12)]
    links += [(0, 3, 5, 1, 3), (3, 3, 0, 0, 0)]
    Fp = oracle.gauge_force_at(U, 1.9, oracle.IWASAKI_C1, links)
    for n, l in enumerate(links):
        assert np.abs(Fp[n] - F[l]).max() < 1e-13
