"""EOFA hybrid Monte Carlo (Section 3), optionally with the gauge action.

H = sum tr P^2 + S_EOFA(U) [+ S_g(U)].  A trajectory draws
phi = M_EOFA^(-1/2) eta by the rational heatbath of eq. (3.1), integrates
the molecular dynamics, and accepts or rejects by Metropolis.  Each fermion
force evaluation is two Cayley-form CG solves plus the eq. (3.2) force
kernel; the momentum and link updates run in FP64 in eofa_md_update.

gauge = (beta, c1) adds the gauge action of Table 1's ensembles (Iwasaki:
c1 = -0.331; Wilson: c1 = 0).  With n_gauge = 0 its force joins the fermion
force at every evaluation (one time scale); with n_gauge >= 1 every link
update U <- exp(i t P) U of the outer integrator becomes n_gauge steps of
the gauge dynamics over t (two time scales: the cheap gauge force on the
fine one), force-gradient steps by default (gauge_scheme) or leapfrog.
Off equilibrium the gauge force is large and its energy error grows with
the volume, so the fourth-order inner step pays for its four gauge-force
evaluations.  The force-gradient displacement then uses the fermion
force only: the gauge force, a function of the links alone, commutes with
it in the step's commutator terms.

The caller draws every random number (eta, the momenta, the Metropolis
uniform); this module draws none.
"""
from __future__ import annotations

import math

from .api import Context


def hamiltonian(ctx: Context, U, P, phi, m1, m2, gauge=None, **solver):
    """(H, S_EOFA, sum tr P^2, solver statistics); H includes S_g when
    gauge = (beta, c1) is given."""
    ctx.update_gauge(U)
    _, _, _, S, st = ctx.eofa_solve(phi, m1, m2, want_mphi=False, **solver)
    kin = ctx.md_update(U, P)            # dt = 0: only the kinetic term
    Sg = ctx.gauge_action(U, *gauge) if gauge is not None else 0.0
    return kin + S + Sg, S, kin, st


class _Forces:
    """Fermion (+ gauge) force evaluations and link updates shared by the
    integrators (see the module docstring for the two gauge schemes)."""

    def __init__(self, ctx, phi, m1, m2, gauge, n_gauge, gauge_scheme, progress, solver):
        if n_gauge < 0:
            raise ValueError("n_gauge must be >= 0")
        if gauge_scheme not in ("force_gradient", "leapfrog"):
            raise ValueError("gauge_scheme is 'force_gradient' or 'leapfrog'")
        self.gauge_scheme = gauge_scheme
        self.Ud = self.Z = None
        self.ctx, self.phi, self.m1, self.m2 = ctx, phi, m1, m2
        self.gauge, self.n_gauge = gauge, int(n_gauge) if gauge is not None else 0
        self.progress, self.solver = progress, solver
        self.stats = []
        self.Fg = None

    def force(self, Ux):
        """Outer force at links Ux: the fermion force, plus the gauge force
        when it lives on the same time scale."""
        ctx = self.ctx
        ctx.update_gauge(Ux)
        F, _, st = ctx.eofa_force(self.m1, self.m2, phi=self.phi, **self.solver)
        if self.gauge is not None and self.n_gauge == 0:
            ctx.gauge_force(Ux, *self.gauge, out=F, accumulate=True)
        self.stats.append(st)
        if self.progress is not None:
            self.progress(len(self.stats) - 1, st)
        return F

    def links(self, U, P, t):
        """U <- exp(i t P) U, or n_gauge leapfrog steps of the gauge
        dynamics over t on the inner time scale."""
        ctx = self.ctx
        if t == 0.0:
            return
        if self.n_gauge == 0:
            ctx.md_update(U, P, None, dt_p=0.0, dt_u=t)
            return
        h = t / self.n_gauge
        if self.Fg is None:
            self.Fg = ctx.gauge_force(U, *self.gauge)
        if self.gauge_scheme == "leapfrog":
            ctx.gauge_force(U, *self.gauge, out=self.Fg)
            for _ in range(self.n_gauge):
                ctx.md_update(U, P, self.Fg, dt_p=0.5 * h, dt_u=h)
                ctx.gauge_force(U, *self.gauge, out=self.Fg)
                ctx.md_update(U, P, self.Fg, dt_p=0.5 * h, dt_u=0.0)
            return
        for _ in range(self.n_gauge):   # force-gradient QPQPQ on the gauge force alone
            ctx.md_update(U, P, None, dt_p=0.0, dt_u=FG_LAMBDA * h)
            self._gauge_kick(U, P, h)
            ctx.md_update(U, P, None, dt_p=0.0, dt_u=(1.0 - 2.0 * FG_LAMBDA) * h)
            self._gauge_kick(U, P, h)
            ctx.md_update(U, P, None, dt_p=0.0, dt_u=FG_LAMBDA * h)

    def _gauge_kick(self, U, P, h):
        """P <- P - (h/2) F_g(U'), U' = exp(-i xi h^2 F_g(U)) U."""
        import torch
        ctx = self.ctx
        if self.Ud is None:
            self.Ud, self.Z = torch.empty_like(U), torch.empty_like(P)
        ctx.gauge_force(U, *self.gauge, out=self.Fg)
        self.Ud.copy_(U)
        self.Z.zero_()
        ctx.md_update(self.Ud, self.Z, self.Fg, dt_p=FG_XI * h * h, dt_u=1.0)
        ctx.gauge_force(self.Ud, *self.gauge, out=self.Fg)
        ctx.md_update(U, P, self.Fg, dt_p=0.5 * h, dt_u=0.0)


def leapfrog(ctx: Context, U, P, phi, m1, m2, n_steps, dt, progress=None, gauge=None, n_gauge=0,
             gauge_scheme="force_gradient", **solver):
    """In-place leapfrog trajectory; returns per-step statistics.
    progress(i, stats), if given, is called after force evaluation i."""
    fs = _Forces(ctx, phi, m1, m2, gauge, n_gauge, gauge_scheme, progress, solver)
    F = fs.force(U)
    ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=0.0)
    fs.links(U, P, dt)
    for step in range(1, n_steps):
        F = fs.force(U)
        ctx.md_update(U, P, F, dt_p=dt, dt_u=0.0)
        fs.links(U, P, dt)
    F = fs.force(U)
    ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=0.0)
    ctx.update_gauge(U)
    return fs.stats


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


def force_gradient(ctx: Context, U, P, phi, m1, m2, n_steps, dt, progress=None, gauge=None, n_gauge=0,
                   gauge_scheme="force_gradient", **solver):
    """In-place force-gradient QPQPQ trajectory of n_steps x dt; returns the
    per-force-evaluation statistics.  progress(i, stats) as in leapfrog."""
    import torch
    fs = _Forces(ctx, phi, m1, m2, gauge, n_gauge, gauge_scheme, progress, solver)

    def kick():
        F = fs.force(U)
        Ud = U.clone()
        Z = torch.zeros_like(P)
        ctx.md_update(Ud, Z, F, dt_p=FG_XI * dt * dt, dt_u=1.0)   # Z = -xi h^2 F, Ud = e^{iZ} U
        ctx.md_update(U, P, fs.force(Ud), dt_p=0.5 * dt, dt_u=0.0)

    fs.links(U, P, FG_LAMBDA * dt)
    for step in range(n_steps):
        kick()
        fs.links(U, P, (1.0 - 2.0 * FG_LAMBDA) * dt)
        kick()
        last = step == n_steps - 1   # adjacent link updates of two steps merge
        fs.links(U, P, (1.0 if last else 2.0) * FG_LAMBDA * dt)
    ctx.update_gauge(U)
    return fs.stats


class HeatbathIntervalError(RuntimeError):
    """phi^dag M_EOFA phi missed eta^dag eta by more than the guard: the
    rational approximation's interval no longer holds M_EOFA's spectrum."""


def trajectory(ctx: Context, U, P, eta, m1, m2, n_steps, dt, lo, hi, n_poles, u_accept=None,
               integrator=None, progress=None, chrono=0, gauge=None, n_gauge=0,
               gauge_scheme="force_gradient", heatbath_guard=None, **solver):
    """One HMC trajectory from links U and fresh momenta P (both updated in
    place; restored on rejection):
    phi = M_EOFA^(-1/2) eta (eq. (3.1), Zolotarev on [lo, hi] with n_poles),
    H0 = sum tr P^2 + S(phi), the molecular dynamics (`integrator`: leapfrog
    (default) or force_gradient), H1, then accept if u_accept < exp(-(H1 - H0)) (always accept
    when u_accept is None).  chrono > 0 starts the molecular-dynamics solves
    from chronological guesses over the last `chrono` solutions (history
    cleared here, since phi is new).  gauge = (beta, c1), n_gauge and
    gauge_scheme add the gauge action (module docstring).  heatbath_guard:
    if given, phi^dag M_EOFA phi = S0 must equal eta^dag eta to this
    relative tolerance (up to the approximation error, the heatbath draws
    phi with exactly that weight), else HeatbathIntervalError is raised
    before any molecular dynamics, with U and P untouched.  Returns a dict
    with H0, dH, accepted, the fermion and gauge actions and the heatbath
    and force statistics."""
    ctx.update_gauge(U)
    phi, hb = ctx.eofa_heatbath(eta, m1, m2, lo=lo, hi=hi, n_poles=n_poles, **solver)
    ctx.chrono(chrono)
    U0, P0 = U.clone(), P.clone()
    H0, S0, K0, _ = hamiltonian(ctx, U, P, phi, m1, m2, gauge=gauge, **solver)
    if heatbath_guard is not None:
        import torch
        ee = float(torch.linalg.vecdot(eta.reshape(-1), eta.reshape(-1)).real)
        if abs(S0 / ee - 1.0) > heatbath_guard:
            raise HeatbathIntervalError(f"phi^dag M phi / eta^dag eta - 1 = {S0 / ee - 1.0:.3e} "
                                        f"exceeds {heatbath_guard:.1e} on [{lo}, {hi}]")
    step = integrator or leapfrog
    st = step(ctx, U, P, phi, m1, m2, n_steps, dt, progress=progress, gauge=gauge, n_gauge=n_gauge,
              gauge_scheme=gauge_scheme, **solver)
    H1, S1, K1, _ = hamiltonian(ctx, U, P, phi, m1, m2, gauge=gauge, **solver)
    dH = H1 - H0
    accepted = True if u_accept is None else bool(u_accept < math.exp(min(0.0, -dH)))
    if not accepted:
        U.copy_(U0)
        P.copy_(P0)
        ctx.update_gauge(U)
    return {"H0": H0, "dH": dH, "S0": S0, "S1": S1, "Sg0": H0 - S0 - K0, "Sg1": H1 - S1 - K1,
            "accepted": accepted, "heatbath": hb, "forces": st}


# ---------------------------------------------------------------------------
# Markov chain with checkpoint and resume
# ---------------------------------------------------------------------------

def _ckpt_paths(d):
    import os
    return os.path.join(d, "links.npy"), os.path.join(d, "state.json")


def save_checkpoint(directory, U, rng, records, interval=None):
    """Write the links, the generator's state, the trajectory records and
    the heatbath interval in use (if any) to `directory` (each file
    replaced atomically, the state file last)."""
    import json
    import os

    import numpy as np
    os.makedirs(directory, exist_ok=True)
    links, state = _ckpt_paths(directory)
    tmp = links + ".tmp.npy"
    np.save(tmp, U.detach().cpu().numpy())
    os.replace(tmp, links)
    doc = {"n_done": len(records), "rng": rng.bit_generator.state, "records": records, "interval": interval}
    with open(state + ".tmp", "w") as fh:
        json.dump(doc, fh)
    os.replace(state + ".tmp", state)


def load_checkpoint(directory, U, rng, with_interval=False):
    """Restore a checkpoint written by save_checkpoint into U (in place) and
    rng; returns the trajectory records, or None if there is none (with
    with_interval: (records, interval) or None)."""
    import json
    import os

    import numpy as np
    import torch
    links, state = _ckpt_paths(directory)
    if not os.path.exists(state):
        return None
    with open(state) as fh:
        doc = json.load(fh)
    arr = np.load(links, allow_pickle=False)
    if tuple(arr.shape) != tuple(U.shape):
        raise ValueError(f"checkpoint links have shape {arr.shape}, expected {tuple(U.shape)}")
    U.copy_(torch.from_numpy(arr).to(U.device))
    if doc["rng"]["bit_generator"] != type(rng.bit_generator).__name__:
        raise ValueError("checkpoint was written with another bit generator")
    rng.bit_generator.state = doc["rng"]
    records = doc["records"]
    if len(records) != doc["n_done"]:
        raise ValueError("inconsistent checkpoint")
    if with_interval:
        return records, doc.get("interval")
    return records


def spectral_interval(ctx: Context, start, m1, m2, n_iter=12, tol=1e-5, margin=0.02, delta=1e-10,
                      **solver):
    """M_EOFA's spectral interval for the heatbath (Section 3.2): Lanczos
    extremes (eofa_meofa_bounds, n_iter steps from `start`, solves to tol)
    widened by their residual bounds and by `margin`, and the fewest
    Zolotarev poles whose relative error on it is below `delta`.
    Returns {"lo", "hi", "n_poles", "delta"}."""
    from .api import rational_inv_sqrt
    tmin, tmax, rmin, rmax, _ = ctx.meofa_bounds(start, m1, m2, n_iter=n_iter, tol=tol, **solver)
    lo = (1.0 - margin) * max(tmin - rmin, 0.5 * tmin)
    hi = (1.0 + margin) * (tmax + rmax)
    n = next(k for k in range(1, 65) if rational_inv_sqrt(lo, hi, k)[3] <= delta)
    return {"lo": lo, "hi": hi, "n_poles": n, "delta": rational_inv_sqrt(lo, hi, n)[3]}


def run_chain(ctx: Context, U, n_traj, draw, rng, m1, m2, n_steps, dt, lo=None, hi=None, n_poles=None,
              checkpoint=None, interval=None, timings=None, **kw):
    """Run the chain up to n_traj trajectories from links U (updated in
    place).  draw(rng) -> (eta, P, u) gives each trajectory's heatbath noise,
    momenta and Metropolis uniform (the caller decides how); rng is a
    numpy Generator.  Every other argument goes to trajectory().  With
    checkpoint (a directory) the links, rng's state, the records and the
    heatbath interval are saved after every trajectory, and an existing
    checkpoint is resumed first, so a stopped chain continues exactly as if
    it had not stopped.

    The heatbath interval is either fixed (lo, hi, n_poles) or, with
    interval = dict(refresh_every=N, guard=g, **spectral_interval options),
    estimated by Lanczos before the first trajectory and reused for N
    trajectories before it is estimated again (M_EOFA's spectrum is narrow
    and moves little between trajectories, Section 3.2).  Every trajectory
    then checks phi^dag M_EOFA phi against eta^dag eta to the relative
    tolerance g (default 1e-6); if that fails, the interval is estimated
    afresh from the current links and the trajectory is repeated with the
    same draws.  timings (a list), if given, receives per trajectory the
    seconds spent on the interval and on the trajectory itself.
    Returns one record per trajectory (dH, acceptance, actions, iterations)."""
    import time
    records, iv = [], None
    if checkpoint is not None:
        got = load_checkpoint(checkpoint, U, rng, with_interval=True)
        if got is not None:
            records, iv = got
    if interval is None:
        if lo is None or hi is None or n_poles is None:
            raise ValueError("give lo, hi and n_poles, or interval=dict(refresh_every=...)")
        iv = {"lo": lo, "hi": hi, "n_poles": n_poles, "since": 0}
    opts = dict(interval or {})
    every = int(opts.pop("refresh_every", 1))
    guard = opts.pop("guard", 1e-6) if interval is not None else None
    solver = {k: kw[k] for k in ("tol", "maxiter", "inner", "reliable_delta") if k in kw}
    solver.pop("tol", None)
    while len(records) < n_traj:
        eta, P, u = draw(rng)
        t_iv = 0.0
        for attempt in range(2):
            if interval is not None and (iv is None or iv["since"] >= every or attempt > 0):
                t0 = time.perf_counter()
                ctx.update_gauge(U)
                iv = dict(spectral_interval(ctx, eta, m1, m2, **opts, **solver), since=0)
                t_iv += time.perf_counter() - t0
            t0 = time.perf_counter()
            try:
                r = trajectory(ctx, U, P, eta, m1, m2, n_steps, dt, iv["lo"], iv["hi"], iv["n_poles"],
                               u_accept=u, heatbath_guard=guard, **kw)
                break
            except HeatbathIntervalError:
                if attempt > 0 or interval is None:
                    raise
        t_traj = time.perf_counter() - t0
        iv["since"] += 1
        records.append({"dH": r["dH"], "accepted": r["accepted"], "S0": r["S0"], "S1": r["S1"],
                        "Sg0": r["Sg0"], "Sg1": r["Sg1"],
                        "heatbath_iters": list(r["heatbath"]["iters"]),
                        "md_iters": [sum(s["iters"][0] for s in r["forces"]),
                                     sum(s["iters"][1] for s in r["forces"])],
                        "interval": [iv["lo"], iv["hi"], iv["n_poles"]]})
        if timings is not None:
            timings.append({"interval_s": t_iv, "trajectory_s": t_traj})
        if checkpoint is not None:
            save_checkpoint(checkpoint, U, rng, records, interval=iv)
    return records
