"""EOFAAction (torch.autograd.Function) and the EOFA molecular dynamics
(Section 3), with and without the gauge action, on the GPU."""
import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import to_dev

pytestmark = pytest.mark.gpu

C1 = din.preset("c1")


@pytest.fixture(scope="module")
def c1():
    from paper_1611_00298_amd import Context
    U = din.random_gauge(C1["L"], C1["eps"], C1["seed_gauge"])
    phi = din.gaussian_4d(C1["L"], C1["seed_phi"])
    lat = oracle.Lattice(C1["L"], C1["Ls"], M5=C1["M5"], alpha=C1["alpha"])
    ctx = Context(C1["L"], C1["Ls"], to_dev(U), M5=C1["M5"], alpha=C1["alpha"])
    yield lat, U, phi, ctx
    ctx.close()


def test_backward_matches_oracle_gradient(c1):
    import torch
    from paper_1611_00298_amd import eofa_action
    lat, U, phi, ctx = c1
    m1, m2 = C1["m1"], C1["m2"]
    Ut = to_dev(U).requires_grad_(True)
    S = eofa_action(Ut, to_dev(phi), ctx, m1, m2, tol=1e-12)
    S.backward()
    chiL, chiR, _, S2, _ = ctx.eofa_solve(to_dev(phi), m1, m2, tol=1e-12)
    assert float(S) == pytest.approx(S2, rel=1e-12)
    _, Gr = oracle.force(lat, U, m1, m2, chiL.cpu().numpy(), chiR.cpu().numpy())
    G = Ut.grad.cpu().numpy()
    assert np.abs(G - Gr).max() <= 1e-9 * np.abs(Gr).max()


def test_backward_directional_derivative(c1):
    """dS along a random complex direction E: central differences versus
    Re sum tr(G^dag E) (torch's convention for a real function of complex U)."""
    import torch
    from paper_1611_00298_amd import eofa_action
    lat, U, phi, ctx = c1
    m1, m2 = C1["m1"], C1["m2"]
    Ut = to_dev(U).requires_grad_(True)
    S = eofa_action(Ut, to_dev(phi), ctx, m1, m2, tol=1e-13)
    S.backward()
    G = Ut.grad.cpu().numpy()
    rng = np.random.default_rng(8)
    E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    d = 1e-6
    Sp = float(eofa_action(to_dev(U + d * E), to_dev(phi), ctx, m1, m2, tol=1e-13))
    Sm = float(eofa_action(to_dev(U - d * E), to_dev(phi), ctx, m1, m2, tol=1e-13))
    fd = (Sp - Sm) / (2 * d)
    an = np.sum(np.conj(G) * E).real
    assert an == pytest.approx(fd, rel=1e-6)
    ctx.update_gauge(to_dev(U))


def run_trajectory(ctx, U0, P0, phi, n_steps, dt, **solver):
    from paper_1611_00298_amd.hmc import hamiltonian, leapfrog
    U, P = to_dev(U0), to_dev(P0)
    H0, _, _, _ = hamiltonian(ctx, U, P, to_dev(phi), C1["m1"], C1["m2"], **solver)
    leapfrog(ctx, U, P, to_dev(phi), C1["m1"], C1["m2"], n_steps, dt, **solver)
    H1, _, _, _ = hamiltonian(ctx, U, P, to_dev(phi), C1["m1"], C1["m2"], **solver)
    return U, P, H1 - H0


def test_leapfrog_reversibility_and_dt2_scaling(c1):
    lat, U0, phi, ctx = c1
    P0 = din.gaussian_momenta(C1["L"], 305)
    # energy violation falls like dt^2 (second-order integrator, correct force)
    _, _, dH1 = run_trajectory(ctx, U0, P0, phi, 5, 0.1, tol=1e-12)
    _, _, dH2 = run_trajectory(ctx, U0, P0, phi, 10, 0.05, tol=1e-12)
    assert abs(dH1) > 1e-6
    assert 2.5 < abs(dH1 / dH2) < 6.0, (dH1, dH2)
    # reversibility: integrate forward, flip the momenta, integrate back
    from paper_1611_00298_amd.hmc import leapfrog
    U, P, _ = run_trajectory(ctx, U0, P0, phi, 10, 0.1, tol=1e-12)
    P.neg_()
    leapfrog(ctx, U, P, to_dev(phi), C1["m1"], C1["m2"], 10, 0.1, tol=1e-12)
    assert np.abs(U.cpu().numpy() - U0).max() < 1e-10
    assert np.abs(-P.cpu().numpy() - P0).max() < 1e-9
    ctx.update_gauge(to_dev(U0))


def test_mixed_precision_trajectory_against_fp64(c1):
    """Mixed-precision solves inside the force: dH and the end point agree
    with the FP64 trajectory to the solver tolerance."""
    lat, U0, phi, ctx = c1
    P0 = din.gaussian_momenta(C1["L"], 306)
    U64, _, dH64 = run_trajectory(ctx, U0, P0, phi, 10, 0.1, tol=1e-12)
    U16, _, dH16 = run_trajectory(ctx, U0, P0, phi, 10, 0.1, tol=1e-10, inner="fp16")
    assert abs(dH16 - dH64) < 1e-6
    assert np.abs(U16.cpu().numpy() - U64.cpu().numpy()).max() < 1e-8
    ctx.update_gauge(to_dev(U0))


def test_force_gradient_dt4_scaling_and_reversibility(c1):
    """The force-gradient QPQPQ integrator (Section 5's integrator family):
    the energy violation falls like dt^4, it beats leapfrog at the same step,
    and it is reversible."""
    from paper_1611_00298_amd.hmc import force_gradient, hamiltonian
    lat, U0, phi, ctx = c1
    P0 = din.gaussian_momenta(C1["L"], 307)
    ph = to_dev(phi)

    def run(n, dt):
        U, P = to_dev(U0), to_dev(P0)
        H0, _, _, _ = hamiltonian(ctx, U, P, ph, C1["m1"], C1["m2"], tol=1e-12)
        st = force_gradient(ctx, U, P, ph, C1["m1"], C1["m2"], n, dt, tol=1e-12)
        H1, _, _, _ = hamiltonian(ctx, U, P, ph, C1["m1"], C1["m2"], tol=1e-12)
        assert len(st) == 4 * n
        return U, P, H1 - H0

    # trajectory length 0.4 (at 0.8 these synthetic fields leave the asymptotic range at dt = 0.2)
    _, _, dH1 = run(2, 0.2)
    _, _, dH2 = run(4, 0.1)
    _, _, dH_lf = run_trajectory(ctx, U0, P0, phi, 4, 0.1, tol=1e-12)
    assert abs(dH2) > 1e-6, (dH1, dH2)
    assert 9.0 < abs(dH1 / dH2) < 28.0, (dH1, dH2)
    assert abs(dH2) < 0.02 * abs(dH_lf), (dH2, dH_lf)
    U, P, _ = run(4, 0.1)
    P.neg_()
    force_gradient(ctx, U, P, ph, C1["m1"], C1["m2"], 4, 0.1, tol=1e-12)
    assert np.abs(U.cpu().numpy() - U0).max() < 1e-10
    assert np.abs(-P.cpu().numpy() - P0).max() < 1e-9
    ctx.update_gauge(to_dev(U0))


def test_hmc_trajectory_heatbath_metropolis(c1):
    """A full trajectory: heatbath (eq. (3.1)) gives S(phi) = eta^dag eta up to
    the approximation error; u = 0 accepts, u > 1 rejects and restores the
    links and momenta exactly."""
    from paper_1611_00298_amd.hmc import force_gradient, trajectory
    lat, U0, phi, ctx = c1
    eta = din.gaussian_4d(C1["L"], 405)
    P0 = din.gaussian_momenta(C1["L"], 308)
    ee = float(np.vdot(eta, eta).real)
    from paper_1611_00298_amd import rational_inv_sqrt
    tmin, tmax, rmin, rmax, _ = ctx.meofa_bounds(to_dev(eta), C1["m1"], C1["m2"], n_iter=30, tol=1e-10,
                                                 inner="fp64")
    lo, hi = 0.98 * (tmin - rmin), 1.02 * (tmax + rmax)
    n_poles = next(n for n in range(1, 40) if rational_inv_sqrt(lo, hi, n)[3] < 1e-9)
    for u, integ in ((0.0, None), (2.0, force_gradient)):
        U, P = to_dev(U0), to_dev(P0)
        r = trajectory(ctx, U, P, to_dev(eta), C1["m1"], C1["m2"], 3, 0.1, lo=lo, hi=hi, n_poles=n_poles,
                       u_accept=u, integrator=integ, tol=1e-11)
        assert abs(r["S0"] / ee - 1) < 1e-7, (r["S0"], ee, lo, hi, n_poles)
        assert abs(r["dH"]) < 1.0   # leapfrog at dt = 0.1 on these fields: |dH| ~ 0.05
        assert r["accepted"] == (u == 0.0)
        if r["accepted"]:
            assert np.abs(U.cpu().numpy() - U0).max() > 1e-3
        else:
            assert np.array_equal(U.cpu().numpy(), U0) and np.array_equal(P.cpu().numpy(), P0)
    ctx.update_gauge(to_dev(U0))


def test_chronological_guesses(c1):
    """eofa_chrono: a repeated solve starts from its own solution; a leapfrog
    trajectory with a history ends where the one without does (to the solver
    tolerance) with fewer iterations."""
    from paper_1611_00298_amd.hmc import leapfrog
    lat, U0, phi, ctx = c1
    ph = to_dev(phi)
    ctx.update_gauge(to_dev(U0))
    ctx.chrono(4)
    chiL, chiR, _, S, st1 = ctx.eofa_solve(ph, C1["m1"], C1["m2"], tol=1e-11)
    chiL2, chiR2, _, S2, st2 = ctx.eofa_solve(ph, C1["m1"], C1["m2"], tol=1e-11)
    assert max(st2["iters"]) <= 0.2 * min(st1["iters"]), (st1["iters"], st2["iters"])
    assert max(st2["true_resid"]) <= 1e-11
    assert S2 == pytest.approx(S, rel=1e-10)
    # other masses: that history is not used; the solve is as from zero and correct
    ctx.chrono(0)
    _, _, _, S3, st3 = ctx.eofa_solve(ph, 0.1, 0.5, tol=1e-11)
    ctx.chrono(4)
    ctx.eofa_solve(ph, C1["m1"], C1["m2"], tol=1e-11)
    _, _, _, S4, st4 = ctx.eofa_solve(ph, 0.1, 0.5, tol=1e-11)
    assert st4["iters"] == st3["iters"] and S4 == pytest.approx(S3, rel=1e-10)
    P0 = din.gaussian_momenta(C1["L"], 309)
    res = {}
    for depth in (0, 6):
        ctx.chrono(depth)
        U, P = to_dev(U0), to_dev(P0)
        st = leapfrog(ctx, U, P, ph, C1["m1"], C1["m2"], 6, 0.05, tol=1e-11)
        res[depth] = (U.cpu().numpy(), sum(sum(x["iters"]) for x in st))
    ctx.chrono(0)
    assert np.abs(res[6][0] - res[0][0]).max() < 1e-8
    assert res[6][1] < 0.8 * res[0][1], (res[0][1], res[6][1])
    ctx.update_gauge(to_dev(U0))


def test_chronological_md_end_point_by_oracle(c1):
    """The leapfrog end point with chronological guesses (depth 6) against a
    CPU replay of the same six steps with the oracle's solves, force (eq.
    (3.2)) and MD update: the history changes the solves' starting points,
    not what they converge to."""
    from paper_1611_00298_amd.hmc import leapfrog
    lat, U0, phi, ctx = c1
    m1, m2, n, dt = C1["m1"], C1["m2"], 6, 0.05
    P0 = din.gaussian_momenta(C1["L"], 309)
    ctx.update_gauge(to_dev(U0))
    ctx.chrono(6)
    U, P = to_dev(U0), to_dev(P0)
    leapfrog(ctx, U, P, to_dev(phi), m1, m2, n, dt, tol=1e-11)
    ctx.chrono(0)

    def force(Ux):
        chiL, chiR, _ = oracle.eofa_chi(lat, Ux, m1, m2, phi, tol=1e-12)
        return oracle.force(lat, Ux, m1, m2, chiL, chiR, want_grad=False)[0]

    Ur, Pr = oracle.md_update(U0, P0, force(U0), 0.5 * dt, dt)
    for _ in range(1, n):
        Ur, Pr = oracle.md_update(Ur, Pr, force(Ur), dt, dt)
    Ur, Pr = oracle.md_update(Ur, Pr, force(Ur), 0.5 * dt, 0.0)
    assert np.abs(U.cpu().numpy() - Ur).max() < 1e-8
    assert np.abs(P.cpu().numpy() - Pr).max() < 1e-8
    assert np.abs(Ur - U0).max() > 1e-3   # the steps moved the links
    ctx.update_gauge(to_dev(U0))


# 16I's gauge coupling (Table 1) with the Iwasaki coefficient
GAUGE = (2.13, oracle.IWASAKI_C1)


def test_force_gradient_with_gauge_action(c1):
    """H = sum tr P^2 + S_EOFA + S_g.  One time scale (gauge force added to
    the fermion force): still fourth order.  Two time scales (gauge force on
    n_gauge inner leapfrog steps): refining the inner level shrinks |dH|, and
    the scheme is reversible."""
    from paper_1611_00298_amd.hmc import force_gradient, hamiltonian
    lat, U0, phi, ctx = c1
    m1, m2 = C1["m1"], C1["m2"]
    P0 = din.gaussian_momenta(C1["L"], 311)
    ph = to_dev(phi)
    U, P = to_dev(U0), to_dev(P0)
    H0, S0, K0, _ = hamiltonian(ctx, U, P, ph, m1, m2, gauge=GAUGE, tol=1e-12)
    assert H0 - S0 - K0 == pytest.approx(oracle.gauge_action(U0, *GAUGE), rel=1e-10)

    def run(n, dt, ng, scheme="force_gradient"):
        U, P = to_dev(U0), to_dev(P0)
        force_gradient(ctx, U, P, ph, m1, m2, n, dt, gauge=GAUGE, n_gauge=ng, gauge_scheme=scheme,
                       tol=1e-12)
        H1, _, _, _ = hamiltonian(ctx, U, P, ph, m1, m2, gauge=GAUGE, tol=1e-12)
        return U, P, H1 - H0

    _, _, d1 = run(2, 0.2, 0)
    _, _, d2 = run(4, 0.1, 0)
    assert abs(d2) > 1e-7 and 9.0 < abs(d1 / d2) < 28.0, (d1, d2)
    # an inner leapfrog's error dominates dH here, and falls with n_gauge
    _, _, e1 = run(2, 0.2, 1, "leapfrog")
    _, _, e4 = run(2, 0.2, 4, "leapfrog")
    assert abs(e4) < 0.25 * abs(e1), (e1, e4)
    U, P, _ = run(2, 0.2, 2)
    P.neg_()
    force_gradient(ctx, U, P, ph, m1, m2, 2, 0.2, gauge=GAUGE, n_gauge=2, tol=1e-12)
    assert np.abs(U.cpu().numpy() - U0).max() < 1e-10
    assert np.abs(-P.cpu().numpy() - P0).max() < 1e-9
    ctx.update_gauge(to_dev(U0))


@pytest.mark.parametrize("scheme", ["force_gradient", "leapfrog"])
def test_nested_gauge_level_matches_a_cpu_replay(c1, scheme):
    """At m1 = m2 the EOFA force vanishes, so the two-time-scale
    force-gradient trajectory is the pure-gauge integration of each
    link-update segment (lambda h, (1 - 2 lambda) h, 2 lambda h, ...,
    lambda h), n_gauge inner steps each: replayed on the CPU with the
    oracle's force and update."""
    from paper_1611_00298_amd.hmc import FG_LAMBDA, FG_XI, force_gradient
    lat, U0, phi, ctx = c1
    P0 = din.gaussian_momenta(C1["L"], 312)
    n, dt, ng = 2, 0.2, 3
    U, P = to_dev(U0), to_dev(P0)
    force_gradient(ctx, U, P, to_dev(phi), 0.3, 0.3, n, dt, gauge=GAUGE, n_gauge=ng, gauge_scheme=scheme,
                   tol=1e-10)
    segs = [FG_LAMBDA * dt]
    for s in range(n):
        segs += [(1 - 2 * FG_LAMBDA) * dt, (1.0 if s == n - 1 else 2.0) * FG_LAMBDA * dt]
    Fg = lambda X: oracle.gauge_force(X, *GAUGE)
    drift = lambda X, Q, t: oracle.md_update(X, Q, Q, 0.0, t)
    Uc, Pc = U0.copy(), P0.copy()
    for t in segs:
        h = t / ng
        for _ in range(ng):
            if scheme == "leapfrog":
                Uc, Pc = oracle.md_update(Uc, Pc, Fg(Uc), 0.5 * h, h)
                Pc = Pc - 0.5 * h * Fg(Uc)
                continue
            for a in (FG_LAMBDA, 1 - 2 * FG_LAMBDA):
                Uc, Pc = drift(Uc, Pc, a * h)
                Ud, _ = oracle.md_update(Uc, np.zeros_like(Pc), Fg(Uc), FG_XI * h * h, 1.0)
                Pc = Pc - 0.5 * h * Fg(Ud)
            Uc, Pc = drift(Uc, Pc, FG_LAMBDA * h)
    assert np.abs(U.cpu().numpy() - Uc).max() < 1e-10
    assert np.abs(P.cpu().numpy() - Pc).max() < 1e-9
    ctx.update_gauge(to_dev(U0))


def test_trajectory_with_gauge_action(c1):
    """A full trajectory with the gauge action on two time scales: the
    heatbath still gives S_EOFA(phi) = eta^dag eta, S_g is reported at both
    ends, and |dH| stays well below 1."""
    from paper_1611_00298_amd import rational_inv_sqrt
    from paper_1611_00298_amd.hmc import force_gradient, trajectory
    lat, U0, phi, ctx = c1
    eta = din.gaussian_4d(C1["L"], 406)
    P0 = din.gaussian_momenta(C1["L"], 313)
    ee = float(np.vdot(eta, eta).real)
    ctx.update_gauge(to_dev(U0))
    tmin, tmax, rmin, rmax, _ = ctx.meofa_bounds(to_dev(eta), C1["m1"], C1["m2"], n_iter=30, tol=1e-10,
                                                 inner="fp64")
    lo, hi = 0.98 * (tmin - rmin), 1.02 * (tmax + rmax)
    n_poles = next(n for n in range(1, 40) if rational_inv_sqrt(lo, hi, n)[3] < 1e-9)
    U, P = to_dev(U0), to_dev(P0)
    r = trajectory(ctx, U, P, to_dev(eta), C1["m1"], C1["m2"], 2, 0.1, lo=lo, hi=hi, n_poles=n_poles,
                   u_accept=0.0, integrator=force_gradient, gauge=GAUGE, n_gauge=4, tol=1e-11)
    assert abs(r["S0"] / ee - 1) < 1e-7
    assert r["Sg0"] == pytest.approx(oracle.gauge_action(U0, *GAUGE), rel=1e-10)
    assert r["Sg1"] == pytest.approx(oracle.gauge_action(U.cpu().numpy(), *GAUGE), rel=1e-10)
    # rough synthetic fields: an inner leapfrog (n_gauge = 4) gave dH = -0.126 here
    assert r["accepted"] and abs(r["dH"]) < 0.5, r["dH"]
    ctx.update_gauge(to_dev(U0))


def _draw_factory(L):
    T = din.gell_mann() / 2
    shape4 = (L[3], L[2], L[1], L[0])

    def draw(rng):
        s = np.sqrt(0.5)
        eta = rng.normal(scale=s, size=shape4 + (4, 3)) + 1j * rng.normal(scale=s, size=shape4 + (4, 3))
        p = rng.standard_normal((4,) + shape4 + (8,))
        P = np.einsum("...a,aij->...ij", p, T)
        return to_dev(eta), to_dev(P), float(rng.random())
    return draw


def test_chain_checkpoint_resume(c1, tmp_path):
    """A chain stopped after 2 trajectories and resumed (new link tensor,
    new generator) ends bit for bit where the uninterrupted chain does."""
    from paper_1611_00298_amd.hmc import force_gradient, run_chain
    lat, U0, phi, ctx = c1
    draw = _draw_factory(C1["L"])
    kw = dict(integrator=force_gradient, gauge=GAUGE, n_gauge=2, chrono=4, tol=1e-10, inner="fp16")
    args = (C1["m1"], C1["m2"], 2, 0.1, 0.5, 5.0, 4)
    Ua = to_dev(U0)
    ra = run_chain(ctx, Ua, 3, draw, np.random.Generator(np.random.PCG64(7)), *args,
                   checkpoint=str(tmp_path / "a"), **kw)
    Ub = to_dev(U0)
    rb = run_chain(ctx, Ub, 2, draw, np.random.Generator(np.random.PCG64(7)), *args,
                   checkpoint=str(tmp_path / "b"), **kw)
    assert rb == ra[:2]
    Uc = to_dev(np.zeros_like(U0))
    rc = run_chain(ctx, Uc, 3, draw, np.random.Generator(np.random.PCG64(12345)), *args,
                   checkpoint=str(tmp_path / "b"), **kw)
    assert rc == ra
    assert np.array_equal(Uc.cpu().numpy(), Ua.cpu().numpy())
    assert len(ra) == 3 and all(abs(r["dH"]) < 1.0 for r in ra)
    ctx.update_gauge(to_dev(U0))


def test_chain_reuses_the_heatbath_interval(c1, tmp_path):
    """run_chain with interval reuse: Lanczos before trajectories 0 and 2
    (refresh_every = 2), none before 1; a stop after 2 trajectories and a
    resume end where the uninterrupted chain does, interval included."""
    from paper_1611_00298_amd.hmc import force_gradient, run_chain
    lat, U0, phi, ctx = c1
    draw = _draw_factory(C1["L"])
    iv = dict(refresh_every=2, n_iter=20, tol=1e-8, guard=1e-6)
    kw = dict(integrator=force_gradient, tol=1e-10, inner="fp16")
    args = (C1["m1"], C1["m2"], 2, 0.1)
    Ua, ta = to_dev(U0), []
    ra = run_chain(ctx, Ua, 3, draw, np.random.Generator(np.random.PCG64(8)), *args, interval=iv,
                   timings=ta, checkpoint=str(tmp_path / "a"), **kw)
    assert [t["interval_s"] > 0 for t in ta] == [True, False, True]
    assert ra[0]["interval"] == ra[1]["interval"] != ra[2]["interval"]
    lo, hi, n = ra[0]["interval"]
    assert 0 < lo < 1.0 < hi and n >= 1
    Ub = to_dev(U0)
    run_chain(ctx, Ub, 2, draw, np.random.Generator(np.random.PCG64(8)), *args, interval=iv,
              checkpoint=str(tmp_path / "b"), **kw)
    rb = run_chain(ctx, Ub, 3, draw, np.random.Generator(np.random.PCG64(8)), *args, interval=iv,
                   checkpoint=str(tmp_path / "b"), **kw)
    assert rb == ra
    assert np.array_equal(Ub.cpu().numpy(), Ua.cpu().numpy())
    ctx.update_gauge(to_dev(U0))


def test_chain_guard_refreshes_a_wrong_interval(c1, tmp_path):
    """A resumed chain whose saved interval does not hold M_EOFA's spectrum
    (here [3, 5]; the spectrum starts near 1) fails the phi^dag M phi check
    of its next heatbath, re-estimates the interval and carries on."""
    from paper_1611_00298_amd.hmc import run_chain, save_checkpoint
    lat, U0, phi, ctx = c1
    draw = _draw_factory(C1["L"])
    rng = np.random.Generator(np.random.PCG64(9))
    U = to_dev(U0)
    save_checkpoint(str(tmp_path), U, rng, [], interval={"lo": 3.0, "hi": 5.0, "n_poles": 6, "since": 0})
    t = []
    r = run_chain(ctx, U, 1, draw, rng, C1["m1"], C1["m2"], 2, 0.1, checkpoint=str(tmp_path), timings=t,
                  interval=dict(refresh_every=100, n_iter=20, tol=1e-8, guard=1e-6), tol=1e-10)
    assert t[0]["interval_s"] > 0
    lo, hi, n = r[0]["interval"]
    assert lo < 1.0 < hi
    assert abs(r[0]["S0"]) > 0
    ctx.update_gauge(to_dev(U0))
