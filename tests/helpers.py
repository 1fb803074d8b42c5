"""Shared test helpers (no method arithmetic)."""
import numpy as np


def to_dev(a, dev="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def region_rel(a, b):
    """Largest relative L2 error over the thin regions of a 5D field
    (s, t, z, y, x, spin, colour) where the boundary terms act: the s-wrap
    slices s = 0 and s = Ls - 1, and the time faces t = 0 and t = Lt - 1,
    each measured against its own norm (an error confined to one of them
    would vanish in the norm of the whole field)."""
    a = np.asarray(a)
    b = np.asarray(b)
    worst = 0.0
    for idx in ((0,), (b.shape[0] - 1,), (slice(None), 0), (slice(None), b.shape[1] - 1)):
        nb = np.linalg.norm(b[idx])
        if nb > 0:
            worst = max(worst, float(np.linalg.norm(a[idx] - b[idx]) / nb))
    return worst


# stated parity bounds for the reduced-precision operator (a few unit roundoffs)
PREC_TOL = {"fp64": 1e-12, "fp32": 1e-6, "fp16": 2e-3, "bf16": 2e-2}


def abelian_flux_field(L, quanta):
    """U(1) links embedded as diag(e^{i th}, e^{-i th}, 1) with a uniform flux
    F_{mu nu} = 2 pi n_{mu nu} / (L_mu L_nu) through every plaquette of each
    plane on the periodic lattice ('t Hooft's twisted construction):
    th_nu(x) = sum_{mu<nu} F_{mu nu} x_mu, and on the last slice x_mu = L_mu - 1
    th_mu also carries -sum_{nu>mu} F_{mu nu} L_mu x_nu."""
    shape4 = (L[3], L[2], L[1], L[0])
    t, z, y, x = np.indices(shape4)
    X = (x, y, z, t)
    F = {}
    th = np.zeros((4,) + shape4)
    for (mu, nu), n in quanta.items():
        F[mu, nu] = 2 * np.pi * n / (L[mu] * L[nu])
        th[nu] += F[mu, nu] * X[mu]
        th[mu] -= np.where(X[mu] == L[mu] - 1, F[mu, nu] * L[mu] * X[nu], 0.0)
    U = np.zeros((4,) + shape4 + (3, 3), dtype=np.complex128)
    U[..., 0, 0] = np.exp(1j * th)
    U[..., 1, 1] = np.exp(-1j * th)
    U[..., 2, 2] = 1.0
    return U, F


def abelian_flux_action(L, F, beta, c1):
    """Closed form of S_g for the uniform-flux field: a loop enclosing flux
    Phi has Re tr W / 3 = (2 cos Phi + 1)/3; a plane holds one plaquette
    (flux F) and two rectangles (flux 2F, both orientations) per site."""
    V = L[0] * L[1] * L[2] * L[3]
    c0 = 1 - 8 * c1
    S = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            f = F.get((mu, nu), 0.0)
            S += c0 * (1 - (2 * np.cos(f) + 1) / 3) + 2 * c1 * (1 - (2 * np.cos(2 * f) + 1) / 3)
    return beta * V * S
