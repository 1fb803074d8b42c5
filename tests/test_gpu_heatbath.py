"""GPU EOFA heatbath (eq. (3.1)) against the CPU oracle: parity with the
oracle's heatbath (the shifted operators inverted as written), against the
exact M_EOFA^(-1/2) on a lattice small enough for dense algebra, the
defining property phi^dag M_EOFA phi = eta^dag eta at a larger size, and the
Lanczos estimate of M_EOFA's spectral interval."""
import ctypes as C

import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import rel, to_dev
from test_oracle_pins import build_M_eofa, dense

pytestmark = pytest.mark.gpu

C1 = din.preset("c1")
C2 = din.preset("c2")


@pytest.fixture(scope="module")
def c1_heatbath():
    L, Ls = C1["L"], C1["Ls"]
    lat = oracle.Lattice(L, Ls, M5=C1["M5"], alpha=C1["alpha"])
    U = din.random_gauge(L, C1["eps"], C1["seed_gauge"])
    eta = din.gaussian_4d(L, 401)
    a0, a, b, delta = oracle.zolotarev_inv_sqrt(0.5, 3.0, 4)
    phi, its = oracle.eofa_heatbath(lat, U, C1["m1"], C1["m2"], eta, a0, a, b, tol=1e-12)
    return dict(lat=lat, U=U, eta=eta, coeffs=(a0, a, b), phi=phi, its=its)


# (inner precision, true-residual tolerance of every solve, bound on |phi - phi_oracle| / |phi|);
# the bound is about kappa(H) times the tolerance.
CASES = [("fp64", 1e-12, 1e-9), ("fp32", 1e-10, 1e-7), ("fp16", 1e-10, 1e-7), ("bf16", 1e-10, 1e-7)]


@pytest.mark.parametrize("inner,tol,bound", CASES, ids=[c[0] for c in CASES])
def test_heatbath_parity_c1(c1_heatbath, inner, tol, bound):
    from paper_1611_00298_amd import Context
    h = c1_heatbath
    with Context(C1["L"], C1["Ls"], to_dev(h["U"]), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        phi, st = ctx.eofa_heatbath(to_dev(h["eta"]), C1["m1"], C1["m2"], coeffs=h["coeffs"], tol=tol,
                                    inner=inner)
    assert st["converged"]
    assert max(st["true_resid"]) <= tol
    assert min(st["iters"]) > 0
    assert rel(phi.cpu().numpy(), h["phi"]) <= bound


def test_heatbath_interval_form_c1(c1_heatbath):
    """Coefficients computed by the library from [lo, hi] and n give the same phi."""
    from paper_1611_00298_amd import Context
    h = c1_heatbath
    with Context(C1["L"], C1["Ls"], to_dev(h["U"]), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        phi, st = ctx.eofa_heatbath(to_dev(h["eta"]), C1["m1"], C1["m2"], lo=0.5, hi=3.0, n_poles=4,
                                    tol=1e-12)
    assert st["delta"] == pytest.approx(oracle.zolotarev_inv_sqrt(0.5, 3.0, 4)[3], rel=1e-6)
    assert rel(phi.cpu().numpy(), h["phi"]) <= 1e-9


@pytest.mark.parametrize("inner", ["fp64", "fp16"])
def test_heatbath_is_inverse_square_root_dense(inner):
    """On 2x2x2x4, Ls = 4, M_EOFA is built densely by the oracle: the GPU phi
    equals M^(-1/2) eta to within the approximation error delta on an
    interval holding the spectrum (Section 3.2)."""
    from paper_1611_00298_amd import Context
    lat = oracle.Lattice((2, 2, 2, 4), 4, M5=1.8, alpha=2.0)
    U = din.random_gauge(lat.L, 0.3, 11)
    m1, m2 = 0.1, 0.6
    H1 = dense(lambda v: oracle.H_op(lat, U, m1, m1, v), lat.shape5)
    H12 = dense(lambda v: oracle.H_op(lat, U, m1, m2, v), lat.shape5)
    M = build_M_eofa(lat, U, m1, m2, H1, H12)
    lam, V = np.linalg.eigh(0.5 * (M + M.conj().T))
    eta = din.gaussian_4d(lat.L, 402)
    e = eta.reshape(-1)
    exact = V @ ((V.conj().T @ e) / np.sqrt(lam))
    with Context(lat.L, lat.Ls, to_dev(U), M5=1.8, alpha=2.0) as ctx:
        for n in (2, 5):
            phi, st = ctx.eofa_heatbath(to_dev(eta), m1, m2, lo=lam[0], hi=lam[-1], n_poles=n,
                                        tol=1e-12 if inner == "fp64" else 1e-11, inner=inner)
            err = np.linalg.norm(phi.cpu().numpy().reshape(-1) - exact) / np.linalg.norm(exact)
            assert err <= st["delta"] * (1 + 1e-6) + 1e-9, (n, err, st)


def test_heatbath_property_c2():
    """phi^dag M_EOFA phi = eta^dag eta (1 + O(delta)) at 16^3x32, Ls = 16,
    with S recomputed by the GPU action (eq. (2.5)) on a fresh solve; the
    interval [0.05, 20] holds the spectrum of M_EOFA with a wide margin."""
    from paper_1611_00298_amd import Context
    L, Ls = C2["L"], C2["Ls"]
    U = din.random_gauge(L, C2["eps"], C2["seed_gauge"])
    eta = din.gaussian_4d(L, 403)
    with Context(L, Ls, to_dev(U), M5=C2["M5"], alpha=C2["alpha"]) as ctx:
        eta_d = to_dev(eta)
        phi, st = ctx.eofa_heatbath(eta_d, C2["m1"], C2["m2"], lo=0.05, hi=20.0, n_poles=10, tol=1e-10,
                                    inner="fp16")
        assert st["converged"] and st["delta"] < 1e-8
        _, _, _, S, st2 = ctx.eofa_solve(phi, C2["m1"], C2["m2"], tol=1e-10, inner="fp16", want_mphi=False)
        # chronological guesses (Section 5.2) against zero guesses: same phi, fewer iterations
        phi0, st0 = ctx.eofa_heatbath(eta_d, C2["m1"], C2["m2"], lo=0.05, hi=20.0, n_poles=10, tol=1e-10,
                                      inner="fp16", forecast=0)
    ee = float(np.vdot(eta, eta).real)
    assert abs(S / ee - 1.0) <= 1e-7, (S, ee, st, st2)
    # and phi is not eta: M_EOFA is not the identity here
    assert rel(phi.cpu().numpy(), eta) > 1e-3
    assert rel(phi.cpu().numpy(), phi0.cpu().numpy()) <= 1e-8
    assert sum(st["iters"]) < 0.8 * sum(st0["iters"]), (st["iters"], st0["iters"])


def test_heatbath_special_cases(c1_heatbath):
    """n_poles = 0 gives alpha0 eta; m1 = m2 (k = 0) gives
    (alpha0 + sum_l alpha_l gamma_l) eta with no solve."""
    from paper_1611_00298_amd import Context
    h = c1_heatbath
    a0, a, b = h["coeffs"]
    with Context(C1["L"], C1["Ls"], to_dev(h["U"]), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        eta_d = to_dev(h["eta"])
        phi, st = ctx.eofa_heatbath(eta_d, C1["m1"], C1["m2"], coeffs=(a0, [], []))
        assert np.array_equal(phi.cpu().numpy(), a0 * h["eta"])
        assert st["iters"] == [0, 0]
        phi, st = ctx.eofa_heatbath(eta_d, 0.3, 0.3, coeffs=(a0, a, b))
        c0 = a0 + sum(al / (1.0 + bl) for al, bl in zip(a, b))
        assert rel(phi.cpu().numpy(), c0 * h["eta"]) <= 1e-15
        assert st["iters"] == [0, 0]


def test_heatbath_errors(c1_heatbath):
    from paper_1611_00298_amd import Context, _lib
    h = c1_heatbath
    a0, a, b = h["coeffs"]
    with Context(C1["L"], C1["Ls"], to_dev(h["U"]), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        eta_d = to_dev(h["eta"])
        for coeffs, m1, m2 in [((a0, [1.0], [-1.0]), 0.04, 1.0), ((a0, [1.0], [float("nan")]), 0.04, 1.0),
                               ((a0, a, b), 1.0, 0.04)]:
            with pytest.raises(_lib.EOFAError) as e:
                ctx.eofa_heatbath(eta_d, m1, m2, coeffs=coeffs)
            assert e.value.code == _lib.EOFA_EINVAL
        # eta and phi may not alias
        sp = _lib.Solver(1e-10, 100, 0, 0.3)
        ca = (C.c_double * 1)(1.0)
        rc = ctx.lib.eofa_heatbath(ctx.handle, 0.04, 1.0, C.c_void_p(eta_d.data_ptr()), 1, 0.5, ca, ca, 0,
                                   C.c_void_p(eta_d.data_ptr()), C.byref(sp), None)
        assert rc == _lib.EOFA_EINVAL
        with pytest.raises(_lib.EOFAError) as e:
            ctx.eofa_heatbath(eta_d, 0.04, 1.0, coeffs=(a0, a, b), forecast=17)
        assert e.value.code == _lib.EOFA_EINVAL
        with pytest.raises(ValueError):
            ctx.eofa_heatbath(eta_d, 0.04, 1.0)
        # a solve that cannot finish: ENOCONV, phi still written, statistics filled
        with pytest.raises(_lib.EOFAError) as e:
            ctx.eofa_heatbath(eta_d, C1["m1"], C1["m2"], coeffs=(a0, a, b), maxiter=3)
        assert e.value.code == _lib.EOFA_ENOCONV
        phi, st = ctx.eofa_heatbath(eta_d, C1["m1"], C1["m2"], coeffs=(a0, a, b), maxiter=3,
                                    allow_noconv=True)
        assert not st["converged"] and st["iters"][0] > 0 and np.isfinite(phi.cpu().numpy()).all()
        # Lanczos steps and history depth out of range
        for n_iter in (1, 201):
            with pytest.raises(_lib.EOFAError) as e:
                ctx.meofa_bounds(eta_d, C1["m1"], C1["m2"], n_iter=n_iter)
            assert e.value.code == _lib.EOFA_EINVAL
        for depth in (-1, 17):
            with pytest.raises(_lib.EOFAError) as e:
                ctx.chrono(depth)
            assert e.value.code == _lib.EOFA_EINVAL


def test_meofa_bounds_dense():
    """Lanczos extremes of M_EOFA (eq. (2.5)) against the dense spectrum:
    Ritz values lie inside it, each residual interval holds an eigenvalue,
    and enough steps resolve both ends."""
    from paper_1611_00298_amd import Context
    lat = oracle.Lattice((2, 2, 2, 4), 4, M5=1.8, alpha=2.0)
    U = din.random_gauge(lat.L, 0.3, 11)
    m1, m2 = 0.1, 0.6
    H1 = dense(lambda v: oracle.H_op(lat, U, m1, m1, v), lat.shape5)
    H12 = dense(lambda v: oracle.H_op(lat, U, m1, m2, v), lat.shape5)
    M = build_M_eofa(lat, U, m1, m2, H1, H12)
    lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
    start = din.gaussian_4d(lat.L, 404)
    with Context(lat.L, lat.Ls, to_dev(U), M5=1.8, alpha=2.0) as ctx:
        for n_iter in (6, 60):
            tmin, tmax, rmin, rmax, st = ctx.meofa_bounds(to_dev(start), m1, m2, n_iter=n_iter, tol=1e-12,
                                                          inner="fp64")
            assert st["converged"] and min(st["iters"]) > 0
            assert lam[0] - 1e-9 <= tmin <= tmax <= lam[-1] + 1e-9
            assert np.abs(lam - tmin).min() <= rmin + 1e-9
            assert np.abs(lam - tmax).min() <= rmax + 1e-9
        # the top of the spectrum is isolated and converges fully; the bottom
        # (M_L's eigenvalues, clustered near 1) to well within what an
        # interval for the rational approximation needs
        assert tmax == pytest.approx(lam[-1], rel=1e-8) and rmax < 1e-6, (tmax, rmax, lam[-3:])
        assert tmin == pytest.approx(lam[0], rel=1e-3), (tmin, rmin, lam[:3])


# ragged workgroup tails, odd Ls, Shamir (alpha = 1) and periodic time
HB_SHAPES = [((4, 2, 6, 4), 5, 2.0, True), ((4, 4, 2, 2), 4, 1.0, False), ((2, 4, 2, 6), 6, 4.0, True)]


@pytest.mark.parametrize("shape", HB_SHAPES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}_a{c[2]}")
def test_heatbath_parity_shapes(shape):
    from paper_1611_00298_amd import Context
    L, Ls, alpha, ap = shape
    m1, m2 = 0.04, 1.0
    lat = oracle.Lattice(L, Ls, M5=1.8, alpha=alpha, antiperiodic_t=ap)
    U = din.random_gauge(L, 0.3, 23)
    eta = din.gaussian_4d(L, 406)
    a0, a, b, _ = oracle.zolotarev_inv_sqrt(0.5, 5.0, 3)
    ref, _ = oracle.eofa_heatbath(lat, U, m1, m2, eta, a0, a, b, tol=1e-12)
    with Context(L, Ls, to_dev(U), M5=1.8, alpha=alpha, antiperiodic_t=ap) as ctx:
        phi, st = ctx.eofa_heatbath(to_dev(eta), m1, m2, coeffs=(a0, a, b), tol=1e-12)
    assert st["converged"]
    assert rel(phi.cpu().numpy(), ref) <= 1e-9
