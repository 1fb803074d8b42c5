"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/eofa.h declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "eofa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_boundary():
    names = declared_functions()
    for required in ("dwf_apply", "eofa_solve", "eofa_force", "eofa_ctx_create",
                     "eofa_ctx_destroy", "eofa_ctx_update_gauge", "eofa_md_update",
                     "eofa_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1611_00298_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared_functions()


def _geom(L=(4, 4, 4, 4), Ls=8):
    from paper_1611_00298_amd._lib import Geom
    return Geom((C.c_int * 4)(*L), Ls, 1.8, 2.0, 1)


@pytest.mark.parametrize("L,Ls", [((3, 4, 4, 4), 8), ((4, 4, 4, 0), 8), ((4, 4, 4, 4), 0),
                                  ((4, 4, 4, 4), 65)])
def test_bad_geometry_is_rejected_on_the_host(L, Ls):
    from paper_1611_00298_amd import _lib
    lib = _lib.load()
    h = C.c_void_p()
    g = _geom(L, Ls)
    dummy = C.c_void_p(1)   # never dereferenced: validation fails first
    rc = lib.eofa_ctx_create(C.byref(h), C.byref(g), dummy, None)
    assert rc == _lib.EOFA_EINVAL
    assert h.value is None
    assert lib.eofa_last_error().decode() != ""


def test_null_arguments_are_rejected():
    from paper_1611_00298_amd import _lib
    lib = _lib.load()
    g = _geom()
    assert lib.eofa_ctx_create(None, C.byref(g), C.c_void_p(1), None) == _lib.EOFA_EINVAL
    assert lib.dwf_apply(None, 0.1, 0.1, 0, 0, 0, None, None) == _lib.EOFA_EINVAL
    sp = _lib.Solver(1e-10, 100, 0, 0.1)
    assert lib.eofa_solve(None, 0.1, 0.2, None, None, None, None, None, None, None,
                          C.byref(sp), None) == _lib.EOFA_EINVAL
    assert lib.eofa_force(None, 0.1, 0.2, None, None, None, None, None, C.byref(sp),
                          None) == _lib.EOFA_EINVAL
    assert lib.eofa_md_update(None, None, None, None, 0.0, 0.0, None) == _lib.EOFA_EINVAL
    assert lib.eofa_md_update_noalloc(None, None, None, None, 0.0, 0.0, None) == _lib.EOFA_EINVAL
    assert lib.eofa_heatbath(None, 0.1, 0.2, None, 0, 1.0, None, None, 0, None, C.byref(sp),
                             None) == _lib.EOFA_EINVAL
    assert lib.eofa_meofa_bounds(None, 0.1, 0.2, None, 10, C.byref(sp), None, None,
                                 None) == _lib.EOFA_EINVAL
    assert lib.eofa_chrono(None, 4) == _lib.EOFA_EINVAL
    assert lib.eofa_solve_dense(None, 0.1, 0.2, None, None, None, None, None, C.byref(sp),
                                None) == _lib.EOFA_EINVAL
    S = C.c_double(0.0)
    assert lib.eofa_gauge_action(None, None, 2.0, -0.331, C.byref(S)) == _lib.EOFA_EINVAL
    assert lib.eofa_gauge_force(None, None, 2.0, -0.331, None, 0) == _lib.EOFA_EINVAL
    lib.eofa_ctx_destroy(None)


@pytest.mark.parametrize("lo,hi,n", [(0.5, 5.0, 3), (0.9, 2.7, 4), (1.0, 100.0, 6), (0.05, 50.0, 10),
                                     (2.0, 2.0, 2), (1e-3, 10.0, 20)])
def test_rational_coefficients_match_the_oracle(lo, hi, n):
    """The library's Zolotarev coefficients (host code, elliptic functions by
    the AGM) against the oracle's (scipy's elliptic functions); the oracle's
    are pinned by the alternation theorem."""
    import numpy as np
    import oracle
    from paper_1611_00298_amd import rational_inv_sqrt
    a0, a, b, delta = rational_inv_sqrt(lo, hi, n)
    o0, oa, ob, od = oracle.zolotarev_inv_sqrt(lo, hi, n)
    assert a0 == pytest.approx(o0, rel=1e-12)
    assert np.allclose(a, oa, rtol=1e-12, atol=0) and np.allclose(b, ob, rtol=1e-12, atol=0)
    assert delta == pytest.approx(od, rel=1e-6, abs=1e-13)


@pytest.mark.parametrize("lo,hi,n", [(0.0, 1.0, 2), (-1.0, 1.0, 2), (2.0, 1.0, 2), (1.0, float("inf"), 2),
                                     (1.0, 2.0, 0), (1.0, 2.0, 65)])
def test_rational_bad_arguments(lo, hi, n):
    from paper_1611_00298_amd import _lib, rational_inv_sqrt
    with pytest.raises(_lib.EOFAError) as e:
        rational_inv_sqrt(lo, hi, n)
    assert e.value.code == _lib.EOFA_EINVAL


def test_product_path_does_not_touch_the_oracle():
    """The product package must not import or load the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1611_00298_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f
