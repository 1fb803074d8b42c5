"""GPU parity of the Moebius operator (eq. (2.3)) and its even-odd Schur
complement (Section 5.1) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import PREC_TOL, region_rel, rel, to_dev

pytestmark = pytest.mark.gpu

# (L, Ls, alpha, antiperiodic): C1 shape, ragged workgroup tails, odd Ls,
# Shamir and alpha = 4, periodic time, and the extremes of Ls (1, 2 and the
# largest the library accepts, 64: 4 sites of 64 slices per workgroup)
CASES = [
    ((4, 4, 4, 4), 8, 2.0, True),
    ((4, 2, 6, 4), 5, 2.0, True),
    ((2, 4, 2, 6), 3, 4.0, True),
    ((4, 4, 2, 2), 16, 1.0, False),
    ((2, 2, 4, 4), 24, 2.0, True),
    ((6, 2, 2, 2), 1, 2.0, True),
    ((2, 2, 2, 4), 2, 2.0, True),
    ((2, 2, 2, 6), 64, 2.0, True),
]
MASSES = [(0.04, 0.04), (0.0362, 1.0)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}_a{c[2]}")
def setup(request):
    from paper_1611_00298_amd import Context
    L, Ls, alpha, ap = request.param
    U = din.random_gauge(L, 0.4, 11)
    psi = din.gaussian_5d(L, Ls, 12)
    lat = oracle.Lattice(L, Ls, M5=1.8, alpha=alpha, antiperiodic_t=ap)
    ctx = Context(L, Ls, to_dev(U), M5=1.8, alpha=alpha, antiperiodic_t=ap)
    yield lat, U, psi, ctx
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("masses", MASSES)
def test_ddwf_parity(setup, prec, dagger, masses):
    lat, U, psi, ctx = setup
    mp, mm = masses
    out = ctx.dwf_apply(to_dev(psi), mp, mm, dagger=dagger, prec=prec).cpu().numpy()
    ref = oracle.ddwf(lat, U, mp, mm, psi, dagger=dagger)
    assert rel(out, ref) < PREC_TOL[prec]
    assert region_rel(out, ref) < PREC_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("masses", MASSES)
def test_schur_parity(setup, prec, dagger, masses):
    lat, U, psi, ctx = setup
    mp, mm = masses
    out = ctx.dwf_apply(to_dev(psi), mp, mm, dagger=dagger, eo=True, prec=prec).cpu().numpy()
    ref = oracle.schur(lat, U, mp, mm, psi, dagger=dagger)
    even = (lat.parity_mask() == 0)[None, ..., None, None]
    assert np.abs(out * even).max() == 0.0
    assert rel(out, ref) < PREC_TOL[prec]
    assert region_rel(out, ref) < PREC_TOL[prec]


def test_adjoint_identity_gpu(setup):
    lat, U, psi, ctx = setup
    x = din.gaussian_5d(lat.L, lat.Ls, 21)
    y = din.gaussian_5d(lat.L, lat.Ls, 22)
    odd = (lat.parity_mask() == 1)[None, ..., None, None]
    for eo in (False, True):
        xx, yy = (x * odd, y * odd) if eo else (x, y)
        Dy = ctx.dwf_apply(to_dev(yy), 0.1, 0.5, eo=eo).cpu().numpy()
        Ddx = ctx.dwf_apply(to_dev(xx), 0.1, 0.5, dagger=True, eo=eo).cpu().numpy()
        lhs, rhs = np.vdot(xx, Dy), np.vdot(Ddx, yy)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_deterministic(setup):
    lat, U, psi, ctx = setup
    a = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, eo=True).cpu().numpy()
    b = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, eo=True).cpu().numpy()
    assert np.array_equal(a, b)


def test_force_parity_shapes(setup):
    """Eq. (3.2) force kernel on every shape above (ragged workgroup tails,
    Ls = 1, periodic time) for arbitrary chi_L, chi_R, against the oracle."""
    lat, U, psi, ctx = setup
    m1, m2 = MASSES[1]
    chiL = psi
    chiR = din.gaussian_5d(lat.L, lat.Ls, 13)
    F, G, _ = ctx.eofa_force(m1, m2, chiL=to_dev(chiL), chiR=to_dev(chiR), want_grad=True)
    Fr, Gr = oracle.force(lat, U, m1, m2, chiL, chiR)
    assert np.abs(F.cpu().numpy() - Fr).max() <= 1e-12 * np.abs(Fr).max()
    assert np.abs(G.cpu().numpy() - Gr).max() <= 1e-12 * np.abs(Gr).max()


@pytest.mark.parametrize("blocks", ["1", "0", "2"])
@pytest.mark.parametrize("tile", ["p2,2,2,2,2,1,t", "p1,2,4,4,2,1,t", "p2,4,1,2,1,2,t", "z,2,1,1,t", "p2,2,1,2,2,1,t",
                                  "q2,1,2,2,1,2,1,1,t", "q1,1,2,4,2,2,2,1,z", "none"])
def test_traversal_layouts(tile, blocks, monkeypatch):
    """The hop's site traversal (the XCD regions and tiles of EOFA_TILE, a
    tuning override; with EOFA_BLOCKS=1, the default, the hops walk whole
    2x2x2x2 blocks and share their inside neighbours through LDS where that
    costs no occupancy, 2 forces the block form, 0 turns it off) only
    reorders the work: D_DWF and Mhat in every precision equal the oracle's
    under every layout, including partitions into fewer than 8 regions
    (which fall back to the natural order), and for workgroups of 1
    (Ls = 24) and 3 (Ls = 8) blocks; at Ls = 8 the forced block form stages
    its links in several batches per work-item."""
    from paper_1611_00298_amd import Context
    monkeypatch.setenv("EOFA_TILE", tile)
    monkeypatch.setenv("EOFA_BLOCKS", blocks)
    for L, Ls in (((4, 8, 8, 16), 8), ((8, 4, 4, 8), 24)):
        U = din.random_gauge(L, 0.4, 31)
        psi = din.gaussian_5d(L, Ls, 32)
        lat = oracle.Lattice(L, Ls, M5=1.8, alpha=2.0)
        ref = oracle.ddwf(lat, U, 0.04, 1.0, psi)
        ref_s = oracle.schur(lat, U, 0.04, 1.0, psi, dagger=True)
        with Context(L, Ls, to_dev(U), M5=1.8, alpha=2.0) as ctx:
            for prec in ("fp64", "fp32", "fp16", "bf16"):
                out = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, prec=prec).cpu().numpy()
                assert rel(out, ref) < PREC_TOL[prec]
                assert region_rel(out, ref) < PREC_TOL[prec]
                out = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, dagger=True, eo=True, prec=prec).cpu().numpy()
                assert rel(out, ref_s) < PREC_TOL[prec]
                assert region_rel(out, ref_s) < PREC_TOL[prec]


@pytest.mark.parametrize("L,Ls", [((4, 4, 4, 4), 8), ((2, 2, 4, 4), 24), ((4, 4, 2, 2), 16)])
def test_gauge_update_reaches_every_link_copy(L, Ls):
    """After eofa_ctx_update_gauge every precision's derived links (the
    FP32 copy, the compact 16-bit links of the matrix-core paths and the
    block-major copies of the block-sharing hops, each built on first use)
    follow the new field: D_DWF and Mhat equal the oracle's on the second
    field, in every precision."""
    from paper_1611_00298_amd import Context
    U1 = din.random_gauge(L, 0.4, 41)
    U2 = din.random_gauge(L, 0.4, 42)
    psi = din.gaussian_5d(L, Ls, 43)
    lat = oracle.Lattice(L, Ls, M5=1.8, alpha=2.0)
    with Context(L, Ls, to_dev(U1), M5=1.8, alpha=2.0) as ctx:
        for prec in ("fp64", "fp32", "fp16", "bf16"):   # build every derived copy on U1
            ctx.dwf_apply(to_dev(psi), 0.04, 1.0, eo=True, prec=prec)
        ctx.update_gauge(to_dev(U2))
        ref = oracle.ddwf(lat, U2, 0.04, 1.0, psi)
        ref_s = oracle.schur(lat, U2, 0.04, 1.0, psi, dagger=True)
        for prec in ("fp64", "fp32", "fp16", "bf16"):
            out = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, prec=prec).cpu().numpy()
            assert rel(out, ref) < PREC_TOL[prec]
            out = ctx.dwf_apply(to_dev(psi), 0.04, 1.0, dagger=True, eo=True, prec=prec).cpu().numpy()
            assert rel(out, ref_s) < PREC_TOL[prec]
