"""Seeded synthetic inputs for the EOFA hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds no part of the method's arithmetic: it only draws random numbers and
shapes them into fields in the natural (lexicographic) layout:

* gauge field  U[mu, t, z, y, x, a, b]          complex128, mu = 0..3 <-> x,y,z,t
* 4D spinor    phi[t, z, y, x, spin, colour]     complex128
* 5D spinor    psi[s, t, z, y, x, spin, colour]  complex128
* momenta      P[mu, t, z, y, x, a, b]           complex128, Hermitian traceless

Links are U = exp(i eps H) with H a random traceless Hermitian 3x3 matrix
(iid N(0,1) real and imaginary parts before projection), exponentiated by
eigen-decomposition.  The paper uses thermalised ensembles (Table 1: 16I,
24ID); only their shapes are reproduced here.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "PRESETS", "preset", "rng", "random_gauge", "random_su3", "gaussian_4d",
    "gaussian_5d", "gaussian_momenta", "gell_mann",
]

# Lattice extents are given as (Lx, Ly, Lz, Lt).
PRESETS = {
    # small correctness case: 4^4 with Ls = 8
    "c1": dict(L=(4, 4, 4, 4), Ls=8, M5=1.8, alpha=2.0, m1=0.04, m2=1.0,
               eps=0.3, seed_gauge=101, seed_phi=201),
    # 16I shape (Table 1): 16^3 x 32, Ls = 16
    "c2": dict(L=(16, 16, 16, 32), Ls=16, M5=1.8, alpha=2.0, m1=0.04, m2=1.0,
               eps=0.5, seed_gauge=102, seed_phi=202),
    # 24ID shape (Table 1): 24^3 x 64, Ls = 24
    "c3": dict(L=(24, 24, 24, 64), Ls=24, M5=1.8, alpha=2.0, m1=0.0362, m2=1.0,
               eps=0.5, seed_gauge=103, seed_phi=203),
    # force / differentiation case, 16I shape
    "c4": dict(L=(16, 16, 16, 32), Ls=16, M5=1.8, alpha=2.0, m1=0.04, m2=1.0,
               eps=0.5, seed_gauge=104, seed_phi=204),
    # short trajectory, 24ID shape
    "c5": dict(L=(24, 24, 24, 64), Ls=24, M5=1.8, alpha=2.0, m1=0.0362, m2=1.0,
               eps=0.5, seed_gauge=105, seed_phi=205, seed_mom=305,
               n_steps=10, dt=0.1),
}


def preset(name: str) -> dict:
    return dict(PRESETS[name])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _shape4(L):
    Lx, Ly, Lz, Lt = L
    return (Lt, Lz, Ly, Lx)


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices, by eigh."""
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def _random_traceless_hermitian(g: np.random.Generator, shape) -> np.ndarray:
    A = g.standard_normal(shape + (3, 3)) + 1j * g.standard_normal(shape + (3, 3))
    H = 0.5 * (A + np.swapaxes(A.conj(), -1, -2))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H -= tr[..., None, None] * np.eye(3)
    return H


def random_su3(shape, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Stack of SU(3) matrices exp(i eps H), H random traceless Hermitian."""
    g = rng(seed)
    n = int(np.prod(shape)) if len(shape) else 1
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        H = _random_traceless_hermitian(g, (hi - lo,))
        out[lo:hi] = _expi_hermitian(H, eps)
    return out.reshape(tuple(shape) + (3, 3))


def random_gauge(L, eps: float, seed: int) -> np.ndarray:
    """Random gauge field U[mu,t,z,y,x,3,3] with links exp(i eps H)."""
    return random_su3((4,) + _shape4(L), eps, seed)


def gaussian_4d(L, seed: int) -> np.ndarray:
    """4D complex Gaussian spinor field, Re and Im ~ N(0, 1/2)."""
    g = rng(seed)
    shp = _shape4(L) + (4, 3)
    s = np.sqrt(0.5)
    return g.normal(scale=s, size=shp) + 1j * g.normal(scale=s, size=shp)


def gaussian_5d(L, Ls: int, seed: int) -> np.ndarray:
    """5D complex Gaussian spinor field psi[s,t,z,y,x,4,3], Re, Im ~ N(0, 1/2)."""
    g = rng(seed)
    shp = (Ls,) + _shape4(L) + (4, 3)
    s = np.sqrt(0.5)
    out = np.empty(shp, dtype=np.complex128)
    out.real = g.normal(scale=s, size=shp)
    out.imag = g.normal(scale=s, size=shp)
    return out


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda^a, shape (8,3,3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def gaussian_momenta(L, seed: int) -> np.ndarray:
    """Momenta P = sum_a p^a T^a with p^a ~ N(0,1) and T^a = lambda^a / 2."""
    g = rng(seed)
    p = g.standard_normal((4,) + _shape4(L) + (8,))
    T = gell_mann() / 2
    return np.einsum("...a,aij->...ij", p, T)
