"""Fermion-only EOFA molecular dynamics (Section 3): leapfrog on (U, P).

H = sum tr P^2 + S_EOFA(U).  Each force evaluation is two Cayley-form CG
solves plus the eq. (3.2) force kernel; the momentum and link updates run
in FP64 in eofa_md_update.
"""
from __future__ import annotations

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
