"""Gauge action of the ensembles (Table 1: Iwasaki; Wilson at c1 = 0) and its
force through the C ABI, against the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import abelian_flux_action, abelian_flux_field, to_dev

pytestmark = pytest.mark.gpu

# (L = (Lx, Ly, Lz, Lt), link spread eps): several blocks of 256 links with a
# ragged last one, a non-cubic box, the smallest lattice (every +-2 offset
# wraps onto the site itself) and a flat one
SHAPES = [((4, 4, 4, 4), 0.5), ((4, 6, 2, 8), 0.8), ((2, 2, 2, 2), 1.0), ((6, 4, 4, 2), 0.3),
          ((8, 2, 6, 4), 0.6)]
C1 = [0.0, oracle.IWASAKI_C1]


def _ctx(L, U):
    import paper_1611_00298_amd as eofa
    return eofa.Context(L, 2, U)


@pytest.mark.parametrize("c1", C1)
@pytest.mark.parametrize("L,eps", SHAPES)
def test_gauge_action_and_force_parity(L, eps, c1):
    U = din.random_gauge(L, eps, 131)
    beta = 2.13
    Ud = to_dev(U)
    ctx = _ctx(L, Ud)
    S = ctx.gauge_action(Ud, beta, c1)
    S_ref = oracle.gauge_action(U, beta, c1)
    assert S == pytest.approx(S_ref, rel=1e-13)
    F = ctx.gauge_force(Ud, beta, c1).cpu().numpy()
    F_ref = oracle.gauge_force(U, beta, c1)
    assert np.abs(F - F_ref).max() <= 1e-13 * np.abs(F_ref).max()
    ctx.close()


@pytest.mark.parametrize("c1", C1)
def test_gauge_force_accumulates(c1):
    L = (4, 4, 2, 6)
    U = din.random_gauge(L, 0.6, 132)
    F0 = din.gaussian_momenta(L, 133)
    Ud = to_dev(U)
    ctx = _ctx(L, Ud)
    out = to_dev(F0)
    ctx.gauge_force(Ud, 1.5, c1, out=out, accumulate=True)
    ref = F0 + oracle.gauge_force(U, 1.5, c1)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("c1", C1)
def test_gauge_unit_field_and_uniform_flux(c1):
    """Unit links: S = F = 0 exactly.  Uniform abelian flux (after a random
    gauge rotation): the closed form of S, and a vanishing force."""
    L = (4, 6, 4, 8)
    shape4 = (L[3], L[2], L[1], L[0])
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), (4,) + shape4 + (3, 3)).copy()
    Ud = to_dev(one)
    ctx = _ctx(L, Ud)
    assert ctx.gauge_action(Ud, 2.0, c1) == 0.0
    assert float(ctx.gauge_force(Ud, 2.0, c1).abs().max()) == 0.0
    quanta = {(0, 1): 1, (0, 2): 2, (0, 3): 3, (1, 2): 1, (1, 3): 5, (2, 3): 2}
    U, Fl = abelian_flux_field(L, quanta)
    g = din.random_su3(shape4, 1.0, 134)
    Ug = np.empty_like(U)
    for mu in range(4):
        ax = (3, 2, 1, 0)[mu]
        Ug[mu] = g @ U[mu] @ np.swapaxes(np.roll(g, -1, axis=ax).conj(), -1, -2)
    Ud = to_dev(Ug)
    V = L[0] * L[1] * L[2] * L[3]
    assert ctx.gauge_action(Ud, 1.7, c1) == pytest.approx(abelian_flux_action(L, Fl, 1.7, c1), rel=1e-12)
    assert float(ctx.gauge_force(Ud, 1.7, c1).abs().max()) < 1e-12 * 1.7 * V
    ctx.close()


def test_gauge_fullsize_24ID_shape():
    """24^3 x 64 (the 24ID shape of Table 1), Iwasaki: the action against the
    whole-lattice oracle, the force at sampled links (boundary ones included)
    against the pointwise oracle."""
    p = din.preset("c3")
    L = p["L"]
    U = din.random_gauge(L, p["eps"], p["seed_gauge"])
    beta = 2.25
    Ud = to_dev(U)
    ctx = _ctx(L, Ud)
    S = ctx.gauge_action(Ud, beta, oracle.IWASAKI_C1)
    F = ctx.gauge_force(Ud, beta, oracle.IWASAKI_C1)
    r = np.random.default_rng(135)
    shape4 = (L[3], L[2], L[1], L[0])
    links = [(int(r.integers(4)),) + tuple(int(r.integers(n)) for n in shape4) for _ in range(40)]
    links += [(mu,) + tuple(n - 1 for n in shape4) for mu in range(4)]
    links += [(mu, 0, 0, 0, 0) for mu in range(4)]
    Fs = np.stack([F[l].cpu().numpy() for l in links])
    F_ref = oracle.gauge_force_at(U, beta, oracle.IWASAKI_C1, links)
    assert np.abs(Fs - F_ref).max() <= 1e-13 * np.abs(F_ref).max()
    S_ref = oracle.gauge_action(U, beta, oracle.IWASAKI_C1)
    assert S == pytest.approx(S_ref, rel=1e-12)
    ctx.close()


def _leapfrog_gauge(ctx, U, P, beta, c1, n, dt):
    F = ctx.gauge_force(U, beta, c1)
    ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=dt)
    for _ in range(n - 1):
        ctx.gauge_force(U, beta, c1, out=F)
        ctx.md_update(U, P, F, dt_p=dt, dt_u=dt)
    ctx.gauge_force(U, beta, c1, out=F)
    return ctx.md_update(U, P, F, dt_p=0.5 * dt, dt_u=0.0)


@pytest.mark.parametrize("c1", C1)
def test_pure_gauge_leapfrog_is_second_order_and_reversible(c1):
    """Molecular dynamics of sum tr P^2 + S_g with the GPU force: |dH| falls
    by about 4 when dt halves, and integrating back with -P returns the
    starting links."""
    L = (4, 4, 4, 4)
    beta = 2.0
    U0 = din.random_gauge(L, 0.4, 136)
    P0 = din.gaussian_momenta(L, 137)
    ctx = _ctx(L, to_dev(U0))
    H0 = oracle.kinetic(P0) + oracle.gauge_action(U0, beta, c1)
    dH = []
    for n, dt in ((5, 0.1), (10, 0.05)):
        U, P = to_dev(U0), to_dev(P0)
        kin = _leapfrog_gauge(ctx, U, P, beta, c1, n, dt)
        dH.append(kin + ctx.gauge_action(U, beta, c1) - H0)
    assert abs(dH[0]) > 1e-4
    assert 3.0 < dH[0] / dH[1] < 5.0
    P.neg_()
    _leapfrog_gauge(ctx, U, P, beta, c1, 10, 0.05)
    assert np.abs(U.cpu().numpy() - U0).max() < 1e-11
    ctx.close()


def test_gauge_bad_arguments():
    import paper_1611_00298_amd as eofa
    from paper_1611_00298_amd import _lib
    L = (4, 4, 4, 4)
    Ud = to_dev(din.random_gauge(L, 0.5, 138))
    ctx = _ctx(L, Ud)
    with pytest.raises(eofa.EOFAError):
        ctx.gauge_action(Ud, float("nan"), -0.331)
    with pytest.raises(eofa.EOFAError):
        ctx.gauge_force(Ud, 2.0, float("inf"))
    with pytest.raises(ValueError):
        ctx.gauge_force(Ud, 2.0, -0.331, accumulate=True)
    lib = _lib.load()
    assert lib.eofa_gauge_force(ctx.handle, Ud.data_ptr(), 2.0, -0.331, Ud.data_ptr(), 0) == _lib.EOFA_EINVAL
    S = C.c_double(0.0)
    assert lib.eofa_gauge_action(ctx.handle, Ud.data_ptr(), 2.0, -0.331, None) == _lib.EOFA_EINVAL
    assert lib.eofa_gauge_action(ctx.handle, None, 2.0, -0.331, C.byref(S)) == _lib.EOFA_EINVAL
    with pytest.raises(ValueError):
        ctx.gauge_action(Ud[:, :2].contiguous(), 2.0)
    ctx.close()
