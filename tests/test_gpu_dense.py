"""The dense D_EOFA comparison path (Table 4, "EOFA (dense)"): the EOFA
systems solved on D_EOFA itself, without the Cayley form, against the
oracle's direct solve of H chi = v."""
import ctypes as C

import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import rel, to_dev

pytestmark = pytest.mark.gpu

C1 = din.preset("c1")


def sources(lat, phi, m1, m2):
    om_m, om_p, k = oracle.omega_k(lat, m1, m2)
    vL, vR = lat.zeros5(), lat.zeros5()
    vL[..., 2:, :] = om_m[:, None, None, None, None, None, None] * phi[None, ..., 2:, :]
    vR[..., :2, :] = om_p[:, None, None, None, None, None, None] * phi[None, ..., :2, :]
    return vL, vR


@pytest.mark.parametrize("inner", ["fp64", "fp32", "fp16"])
def test_dense_solve_c1(inner):
    """chi against the oracle's direct (non-Cayley, no even-odd) CGNR on H,
    the true residual recomputed by the oracle, the action, and agreement
    with the GPU's own Cayley-form solve."""
    from paper_1611_00298_amd import Context
    L, Ls, m1, m2 = C1["L"], C1["Ls"], C1["m1"], C1["m2"]
    U = din.random_gauge(L, C1["eps"], C1["seed_gauge"])
    phi = din.gaussian_4d(L, C1["seed_phi"])
    lat = oracle.Lattice(L, Ls, M5=C1["M5"], alpha=C1["alpha"])
    refL, refR, _ = oracle.eofa_chi(lat, U, m1, m2, phi, method="direct", tol=1e-13)
    S_ref, _, M_ref = oracle.action(lat, m1, m2, phi, refL, refR)
    with Context(L, Ls, to_dev(U), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        chiL, chiR, Mphi, S, st = ctx.eofa_solve_dense(to_dev(phi), m1, m2, tol=1e-10, inner=inner)
        cL, cR, _, Sc, stc = ctx.eofa_solve(to_dev(phi), m1, m2, tol=1e-10, inner="fp64")
    chiL, chiR, Mphi = chiL.cpu().numpy(), chiR.cpu().numpy(), Mphi.cpu().numpy()
    assert st["converged"] and min(st["iters"]) > 0 and st["inner_used"] == [inner, inner]
    if inner == "fp64":
        assert st["reliable_updates"] == [0, 0]
    else:
        assert min(st["reliable_updates"]) >= 1
    vL, vR = sources(lat, phi, m1, m2)
    resL = rel(oracle.H_op(lat, U, m1, m1, chiL), vL)
    resR = rel(oracle.H_op(lat, U, m1, m2, chiR), vR)
    assert resL <= 1e-10 and resR <= 1e-10, (resL, resR, st)
    assert abs(st["true_resid"][0] - resL) <= 0.05 * resL + 1e-14
    assert rel(chiL, refL) < 1e-8 and rel(chiR, refR) < 1e-8
    assert abs(S - S_ref) <= 1e-10 * abs(S_ref)
    S2, _, M2 = oracle.action(lat, m1, m2, phi, chiL, chiR)
    assert abs(S - S2) <= 1e-13 * abs(S2) and rel(Mphi, M2) < 1e-13
    assert rel(chiL, cL.cpu().numpy()) < 1e-8 and rel(chiR, cR.cpu().numpy()) < 1e-8
    assert abs(S - Sc) <= 1e-10 * abs(Sc)


SHAPES = [((4, 2, 6, 4), 5, 2.0, True), ((2, 4, 2, 6), 3, 4.0, True), ((4, 4, 2, 2), 4, 1.0, False),
          ((2, 2, 4, 2), 1, 2.0, True), ((4, 4, 4, 2), 16, 2.0, True)]


@pytest.mark.parametrize("inner", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}_a{c[2]}")
def test_dense_solve_shapes(shape, inner):
    """Ragged workgroup tails, odd and single-slice Ls, Shamir (alpha = 1),
    periodic time: the oracle's residual and action."""
    from paper_1611_00298_amd import Context
    L, Ls, alpha, ap = shape
    m1, m2 = 0.04, 1.0
    U = din.random_gauge(L, 0.3, 21)
    phi = din.gaussian_4d(L, 22)
    lat = oracle.Lattice(L, Ls, M5=1.8, alpha=alpha, antiperiodic_t=ap)
    with Context(L, Ls, to_dev(U), M5=1.8, alpha=alpha, antiperiodic_t=ap) as ctx:
        chiL, chiR, _, S, st = ctx.eofa_solve_dense(to_dev(phi), m1, m2, tol=1e-10, inner=inner,
                                                    want_mphi=False)
    assert st["converged"], st
    vL, vR = sources(lat, phi, m1, m2)
    resL = rel(oracle.H_op(lat, U, m1, m1, chiL.cpu().numpy()), vL)
    resR = rel(oracle.H_op(lat, U, m1, m2, chiR.cpu().numpy()), vR)
    assert resL <= 1e-10 and resR <= 1e-10, (resL, resR, st)
    S2, _, _ = oracle.action(lat, m1, m2, phi, chiL.cpu().numpy(), chiR.cpu().numpy())
    assert abs(S - S2) <= 1e-13 * abs(S2)


def test_dense_zero_source_and_errors():
    from paper_1611_00298_amd import Context, _lib
    from paper_1611_00298_amd.api import make_solver
    L, Ls = (4, 4, 4, 4), 4
    U = to_dev(din.random_gauge(L, 0.3, 23))
    with Context(L, Ls, U) as ctx:
        phi = to_dev(np.zeros((4, 4, 4, 4, 4, 3), dtype=np.complex128))
        chiL, chiR, _, S, st = ctx.eofa_solve_dense(phi, 0.1, 0.5)
        assert st["converged"] and st["iters"] == [0, 0] and S == 0.0
        assert float(chiL.abs().max()) == 0.0 and float(chiR.abs().max()) == 0.0
        lib = _lib.load()
        phi = to_dev(din.gaussian_4d(L, 24))
        out = [to_dev(np.zeros((Ls, 4, 4, 4, 4, 4, 3), dtype=np.complex128)) for _ in range(2)]
        S = C.c_double(0.0)
        for inner in ("bf16",):
            sp = make_solver(1e-10, 100, inner, 0.3)
            rc = lib.eofa_solve_dense(ctx.handle, 0.1, 0.5, phi.data_ptr(), out[0].data_ptr(),
                                      out[1].data_ptr(), None, C.byref(S), C.byref(sp), None)
            assert rc == _lib.EOFA_EINVAL
        sp = make_solver(1e-10, 100, "fp64", 0.3)
        rc = lib.eofa_solve_dense(ctx.handle, 0.5, 0.1, phi.data_ptr(), out[0].data_ptr(), out[1].data_ptr(),
                                  None, C.byref(S), C.byref(sp), None)
        assert rc == _lib.EOFA_EINVAL   # m1 > m2
        # maxiter too small: not converged, statistics still written
        _, _, _, _, st = ctx.eofa_solve_dense(phi, 0.1, 0.5, tol=1e-12, maxiter=3, allow_noconv=True)
        assert not st["converged"] and st["iters"] == [3, 3]


def test_dense_fp16_progress_guard():
    """With reliable updates switched off (delta = 1e-30) the FP16 recursion
    loses track of the true residual; the progress guard still forces FP64
    residual recomputations, and the solve ends at the requested true
    residual (in FP16, or after continuing in FP32 or FP64, as reported)."""
    from paper_1611_00298_amd import Context
    L, Ls, m1, m2 = C1["L"], C1["Ls"], C1["m1"], C1["m2"]
    U = din.random_gauge(L, C1["eps"], C1["seed_gauge"])
    phi = din.gaussian_4d(L, C1["seed_phi"])
    lat = oracle.Lattice(L, Ls, M5=C1["M5"], alpha=C1["alpha"])
    with Context(L, Ls, to_dev(U), M5=C1["M5"], alpha=C1["alpha"]) as ctx:
        chiL, chiR, _, S, st = ctx.eofa_solve_dense(to_dev(phi), m1, m2, tol=1e-10, inner="fp16",
                                                    reliable_delta=1e-30, maxiter=40000, want_mphi=False)
    print(f"dense fp16 guard: iters {st['iters']} reliable {st['reliable_updates']} inner {st['inner_used']}")
    assert st["converged"] and min(st["reliable_updates"]) >= 1
    assert all(p in ("fp16", "fp32", "fp64") for p in st["inner_used"])
    vL, vR = sources(lat, phi, m1, m2)
    assert rel(oracle.H_op(lat, U, m1, m1, chiL.cpu().numpy()), vL) <= 1e-10
    assert rel(oracle.H_op(lat, U, m1, m2, chiR.cpu().numpy()), vR) <= 1e-10
