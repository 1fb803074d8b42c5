"""The differentiation and trajectory workloads at their stated sizes.

* 16^3x32, Ls = 16 (the 16I shape of Table 1): the pseudofermion force of
  eq. (3.2) against central finite differences of S = phi^dag M_EOFA phi
  under SU(3) link perturbations U -> exp(+-i delta T^a) U, delta = 1e-5,
  FP64 solves.
* 24^3x64, Ls = 24 (the 24ID shape): a shortened fermion-only leapfrog
  trajectory (Section 3), mixed-precision solves against FP64 ones: the
  energy change, the end point and reversibility.
"""
import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4():
    from paper_1611_00298_amd import Context
    pre = din.preset("c4")
    U = din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"])
    phi = din.gaussian_4d(pre["L"], pre["seed_phi"])
    lat = oracle.Lattice(pre["L"], pre["Ls"], M5=pre["M5"], alpha=pre["alpha"])
    ctx = Context(pre["L"], pre["Ls"], to_dev(U), M5=pre["M5"], alpha=pre["alpha"])
    yield pre, lat, U, phi, ctx
    ctx.close()


def _su3_fd(ctx, U, Ud, ph, phi, m1, m2, mu, site, a, delta, x0):
    """(S(U+) - S(U-)) / (2 delta) for U_mu(x) -> exp(+-i delta T^a) U_mu(x),
    with the difference of the two actions taken site by site as
    Re phi^dag (M_EOFA phi(U+) - M_EOFA phi(U-)), so that their common part
    cancels before the sum over the lattice.  Both FP64 solves start from the
    unperturbed solutions x0 and run to a true residual of 1e-13."""
    T = din.gell_mann() / 2
    Mphi = []
    for sgn in (1.0, -1.0):
        Up = Ud.clone()
        Up[(mu,) + site] = to_dev(oracle.expi_hermitian(sgn * delta * T[a]) @ U[(mu,) + site])
        ctx.update_gauge(Up)
        _, _, M, _, st = ctx.eofa_solve(ph, m1, m2, x0=x0, tol=1e-13, maxiter=50000, want_mphi=True)
        assert st["converged"]
        Mphi.append(M.cpu().numpy())
    ctx.update_gauge(Ud)
    return np.vdot(phi, Mphi[0] - Mphi[1]).real / (2 * delta)


def test_c4_force_finite_differences_local_source(c4):
    """Eq. (3.2) against central finite differences at 16^3x32, Ls = 16,
    m1 = 0.04, m2 = 1, delta = 1e-5, FP64, for 20 random (x, mu, a): the
    force kernel's d^a S = 2 tr(T^a F_mu(x)) agrees to 1e-5 relative.
    Each triple uses a Gaussian pseudofermion supported on the 4^4 block of
    sites around its link, so that S is O(10^3): the FP64 rounding floor of
    S (a few ulps of S, divided by 2 delta) then lies far below 1e-5 of the
    derivative, and the check tests the force and not the arithmetic."""
    pre, lat, U, phi_g, ctx = c4
    m1, m2, delta = pre["m1"], pre["m2"], 1e-5
    Ud = to_dev(U)
    T = din.gell_mann() / 2
    rng = np.random.default_rng(405)
    t_, z_, y_, x_ = np.indices(lat.shape4)
    errs = []
    for i in range(20):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in lat.shape4)
        a = int(rng.integers(8))
        near = np.ones(lat.shape4, dtype=bool)
        for ax, c, n in zip((t_, z_, y_, x_), site, lat.shape4):   # offsets -2..1 (periodic)
            near &= ((ax - c + 2) % n) < 4
        phi = np.where(near[..., None, None], phi_g, 0.0)
        ph = to_dev(phi)
        chiL, chiR, _, _, st = ctx.eofa_solve(ph, m1, m2, tol=1e-13, maxiter=50000, want_mphi=False)
        assert st["converged"]
        F, _, _ = ctx.eofa_force(m1, m2, chiL=chiL, chiR=chiR)
        an = 2 * np.trace(T[a] @ F[(mu,) + site].cpu().numpy()).real
        fd = _su3_fd(ctx, U, Ud, ph, phi, m1, m2, mu, site, a, delta, (chiL, chiR))
        errs.append(abs(fd - an) / abs(an))
        print(f"c4 local FD {i}: mu={mu} site={site} a={a}: analytic {an:+.10e} fd {fd:+.10e} "
              f"rel {errs[-1]:.1e}", flush=True)
        assert abs(an) > 1e-4
    assert max(errs) <= 1e-5, max(errs)


def test_c4_force_finite_differences_gaussian_source(c4):
    """The same check with the Gaussian pseudofermion on the whole 16^3x32
    lattice (S ~ 1.6e6) at delta = 1e-5.  Here S is known only to its FP64
    rounding floor: solves at their floor (true residual ~5e-14) leave a
    non-smooth error of order 1e-15 S in each action, which the difference
    divides by 2 delta.  The bound is 1e-5 relative plus
    1e-14 S / (2 delta) (about 8e-4 here, against force components of
    0.005 to 0.2); the local-source test above makes the 1e-5 check."""
    pre, lat, U, phi, ctx = c4
    m1, m2, delta = pre["m1"], pre["m2"], 1e-5
    Ud, ph = to_dev(U), to_dev(phi)
    ctx.update_gauge(Ud)
    chiL, chiR, _, S0, st = ctx.eofa_solve(ph, m1, m2, tol=1e-13, maxiter=50000, want_mphi=False)
    assert st["converged"]
    F, _, _ = ctx.eofa_force(m1, m2, chiL=chiL, chiR=chiR)
    F = F.cpu().numpy()
    T = din.gell_mann() / 2
    rng = np.random.default_rng(404)
    floor = 1e-14 * abs(S0) / (2 * delta)
    worst = 0.0
    for i in range(20):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in lat.shape4)
        a = int(rng.integers(8))
        fd = _su3_fd(ctx, U, Ud, ph, phi, m1, m2, mu, site, a, delta, (chiL, chiR))
        an = 2 * np.trace(T[a] @ F[(mu,) + site]).real
        worst = max(worst, abs(fd - an) / (1e-5 * abs(an) + floor))
        print(f"c4 FD {i}: mu={mu} site={site} a={a}: analytic {an:+.10e} fd {fd:+.10e}", flush=True)
    print(f"c4 FD: S = {S0:.6e}, floor 1e-14 S/(2 delta) = {floor:.2e}, worst error / bound = {worst:.3f}")
    assert worst <= 1.0


@pytest.fixture(scope="module")
def c5():
    import torch
    from paper_1611_00298_amd import Context
    pre = din.preset("c5")
    U0 = to_dev(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    phi = to_dev(din.gaussian_4d(pre["L"], pre["seed_phi"]))
    P0 = to_dev(din.gaussian_momenta(pre["L"], pre["seed_mom"]))
    ctx = Context(pre["L"], pre["Ls"], U0, M5=pre["M5"], alpha=pre["alpha"])
    yield pre, U0, phi, P0, ctx
    ctx.close()
    del U0, phi, P0
    torch.cuda.empty_cache()


def test_c5_short_trajectory_mixed_vs_fp64(c5):
    """Two leapfrog steps of dt = 0.1 at 24^3x64, Ls = 24 with FP16-inner
    solves against the same steps with FP64 solves (every solve to a true
    residual of 1e-10): equal energy change and end point; the mixed run
    retraced with flipped momenta returns to its start.  The starting
    kinetic energy is the oracle's."""
    from paper_1611_00298_amd.hmc import hamiltonian, leapfrog
    pre, U0, phi, P0, ctx = c5
    m1, m2, dt, n = pre["m1"], pre["m2"], pre["dt"], 2
    res = {}
    for label, solver in (("mixed", dict(tol=1e-10, inner="fp16", reliable_delta=0.3)),
                          ("fp64", dict(tol=1e-10, inner="fp64"))):
        print(f"c5 trajectory: {label}", flush=True)
        U, P = U0.clone(), P0.clone()
        H0, S0, K0, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
        leapfrog(ctx, U, P, phi, m1, m2, n, dt, **solver)
        H1, _, _, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
        res[label] = dict(H0=H0, dH=H1 - H0, K0=K0, U=U, P=P)
        print(f"c5 trajectory {label}: H0 {H0:.10f} dH {H1 - H0:.10e}", flush=True)
        if label == "mixed":
            Ub, Pb = U.clone(), -P
            leapfrog(ctx, Ub, Pb, phi, m1, m2, n, dt, **solver)
            dU, dP = float((Ub - U0).abs().max()), float((Pb + P0).abs().max())
            print(f"c5 trajectory reversed: |dU| {dU:.3e} |dP| {dP:.3e}", flush=True)
            assert dU < 1e-9 and dP < 1e-9
            del Ub, Pb
    mx, fp = res["mixed"], res["fp64"]
    assert mx["K0"] == pytest.approx(oracle.kinetic(P0.cpu().numpy()), rel=1e-12)
    assert abs(mx["H0"] - fp["H0"]) <= 1e-9 * abs(fp["H0"])
    assert abs(fp["dH"]) > 1.0   # the steps move the system: a real energy change to compare
    assert abs(mx["dH"] - fp["dH"]) <= 1e-9 * abs(fp["H0"]) + 1e-6 * abs(fp["dH"])
    assert float((mx["U"] - fp["U"]).abs().max()) < 1e-9
    assert float((mx["P"] - fp["P"]).abs().max()) < 1e-8
    ctx.update_gauge(U0)
