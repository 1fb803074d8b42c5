"""Fermion-only EOFA hybrid Monte Carlo (Section 3).

H = sum tr P^2 + S_EOFA(U).  A trajectory draws phi = M_EOFA^(-1/2) eta by
the rational heatbath of eq. (3.1), integrates the molecular dynamics, and
accepts or rejects by Metropolis.  Each force evaluation is two Cayley-form
CG solves plus the eq. (3.2) force kernel; the momentum and link updates
run in FP64 in eofa_md_update.  The caller draws every random number
(eta, the momenta, the Metropolis uniform); this module draws none.
"""
from __future__ import annotations

import math

from .api import Context


def hamiltonian(ctx: Context, U, P, phi, m1, m2, **solver):
    ctx.update_gauge(U)
    _, _, _, S, st = ctx.eofa_solve(phi, m1, m2, want_mphi=False, **solver)
    kin = ctx.md_update(U, P)            # dt = 0: only the kinetic term
    return kin + S, S, kin, st


def leapfrog(ctx: Context, U, P, phi, m1, m2, n_steps, dt, progress=None, **solver):
    """In-place leapfrog trajectory; returns per-step statistics.
    progress(i, stats), if given, is called after force evaluation i."""
    stats = []

    def force():
        ctx.update_gauge(U)
        F, _, st = ctx.eofa_force(m1, m2, phi=phi, **solver)
        stats.append(st)
        if progress is not None:
            progress(len(stats) - 1, st)
        return F

    F = force()
    ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=dt)
    for step in range(1, n_steps):
        F = force()
        ctx.md_update(U, P, F, dt_p=dt, dt_u=dt)
    F = force()
    ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=0.0)
    ctx.update_gauge(U)
    return stats


# Force-gradient QPQPQ step (the integrator family of Section 5):
#   U <- e^{i lam h P} U;  P <- P - (h/2) F~;  U <- e^{i (1 - 2 lam) h P} U;
#   P <- P - (h/2) F~;  U <- e^{i lam h P} U,
# with F~ = F(U') at links moved along the force, U' = exp(-i xi h^2 F(U)) U.
# In p^a coordinates (H = sum_a (p^a)^2 / 2 + S) the one-step error of this
# symmetric scheme is h^3 (k1 [A,[A,B]] + k2 [B,[A,B]]) + O(h^5) (A the link
# flow, B the momentum flow).  k1 vanishes for lam = (3 - sqrt 3)/6, leaving
# k2 = -(2 - sqrt 3)/24; a kick of weight h/2 with the displaced force adds
# (xi / 4) h^3 [B,[A,B]] (since F(q - e F) = F - (e/2) grad |F|^2), so the
# two kicks cancel k2 for xi = (2 - sqrt 3)/12: fourth order, four force
# evaluations per step.
FG_LAMBDA = (3.0 - math.sqrt(3.0)) / 6.0
FG_XI = (2.0 - math.sqrt(3.0)) / 12.0


def force_gradient(ctx: Context, U, P, phi, m1, m2, n_steps, dt, progress=None, **solver):
    """In-place force-gradient QPQPQ trajectory of n_steps x dt; returns the
    per-force-evaluation statistics.  progress(i, stats) as in leapfrog."""
    import torch
    stats = []

    def force(Ux):
        ctx.update_gauge(Ux)
        F, _, st = ctx.eofa_force(m1, m2, phi=phi, **solver)
        stats.append(st)
        if progress is not None:
            progress(len(stats) - 1, st)
        return F

    def kick():
        F = force(U)
        Ud = U.clone()
        Z = torch.zeros_like(P)
        ctx.md_update(Ud, Z, F, dt_p=FG_XI * dt * dt, dt_u=1.0)   # Z = -xi h^2 F, Ud = e^{iZ} U
        ctx.md_update(U, P, force(Ud), dt_p=0.5 * dt, dt_u=0.0)

    ctx.md_update(U, P, None, dt_p=0.0, dt_u=FG_LAMBDA * dt)
    for step in range(n_steps):
        kick()
        ctx.md_update(U, P, None, dt_p=0.0, dt_u=(1.0 - 2.0 * FG_LAMBDA) * dt)
        kick()
        last = step == n_steps - 1   # adjacent link updates of two steps merge
        ctx.md_update(U, P, None, dt_p=0.0, dt_u=(1.0 if last else 2.0) * FG_LAMBDA * dt)
    ctx.update_gauge(U)
    return stats


def trajectory(ctx: Context, U, P, eta, m1, m2, n_steps, dt, lo, hi, n_poles, u_accept=None,
               integrator=None, progress=None, chrono=0, **solver):
    """One HMC trajectory from links U and fresh momenta P (both updated in
    place; restored on rejection):
    phi = M_EOFA^(-1/2) eta (eq. (3.1), Zolotarev on [lo, hi] with n_poles),
    H0 = sum tr P^2 + S(phi), the molecular dynamics (`integrator`: leapfrog
    (default) or force_gradient), H1, then accept if u_accept < exp(-(H1 - H0)) (always accept
    when u_accept is None).  chrono > 0 starts the molecular-dynamics solves
    from chronological guesses over the last `chrono` solutions (history
    cleared here, since phi is new).  Returns a dict with H0, dH, accepted
    and the heatbath and force statistics."""
    ctx.update_gauge(U)
    phi, hb = ctx.eofa_heatbath(eta, m1, m2, lo=lo, hi=hi, n_poles=n_poles, **solver)
    ctx.chrono(chrono)
    U0, P0 = U.clone(), P.clone()
    H0, S0, _, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
    step = integrator or leapfrog
    st = step(ctx, U, P, phi, m1, m2, n_steps, dt, progress=progress, **solver)
    H1, S1, _, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
    dH = H1 - H0
    accepted = True if u_accept is None else bool(u_accept < math.exp(min(0.0, -dH)))
    if not accepted:
        U.copy_(U0)
        P.copy_(P0)
        ctx.update_gauge(U)
    return {"H0": H0, "dH": dH, "S0": S0, "S1": S1, "accepted": accepted, "heatbath": hb,
            "forces": st}
