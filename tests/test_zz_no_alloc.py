"""The allocation-free MD update (eofa_md_update_noalloc) against
eofa_md_update, through the C ABI: the same links, momenta and kinetic
energy, on two calls in a row of which the second is smaller (the static
scratch array then still holds the first call's partial sums), and the
size limit of that array."""
import numpy as np
import pytest

import dwf_inputs as din
import oracle
from helpers import to_dev

pytestmark = pytest.mark.gpu

MAX_SITES = 16384 * 64   # 128 KiB of partial sums, one per 256 links


def _identity_links(L):
    import torch
    Lx, Ly, Lz, Lt = L
    U = torch.zeros((4, Lt, Lz, Ly, Lx, 3, 3), dtype=torch.complex128, device="cuda")
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def test_noalloc_md_update_matches_md_update():
    import torch
    from paper_1611_00298_amd import Context
    kin = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    # the largest lattice the scratch array serves, then a much smaller one
    for L, seed, random_links in (((32, 32, 32, 32), 501, False), ((6, 4, 4, 8), 511, True)):
        assert L[0] * L[1] * L[2] * L[3] <= MAX_SITES
        print(f"noalloc md update: L={L} seed={seed}", flush=True)
        U0 = to_dev(din.random_gauge(L, 0.5, seed)) if random_links else _identity_links(L)
        P0 = to_dev(din.gaussian_momenta(L, seed + 1))
        F = to_dev(din.gaussian_momenta(L, seed + 2))
        dt_p, dt_u = 0.11, 0.07
        with Context(L, 4, U0) as ctx:
            U1, P1 = U0.clone(), P0.clone()
            k_ref = ctx.md_update(U1, P1, F, dt_p, dt_u)
            U2, P2 = U0.clone(), P0.clone()
            kin.fill_(float("nan"))
            ctx.md_update_noalloc(U2, P2, F, dt_p, dt_u, kinetic=kin)
            torch.cuda.synchronize()
            # the same kernels in the same order: identical results
            assert torch.equal(U2, U1)
            assert torch.equal(P2, P1)
            assert kin.item() == k_ref
            # and the kinetic energy of the updated momenta is the oracle's
            k_orc = oracle.kinetic(P1.cpu().numpy())
            assert k_ref == pytest.approx(k_orc, rel=1e-12)
            # without a kinetic output, and with only one half of the update
            U3, P3 = U0.clone(), P0.clone()
            ctx.md_update_noalloc(U3, P3, F, dt_p, 0.0)
            U4, P4 = U0.clone(), P0.clone()
            ctx.md_update(U4, P4, F, dt_p, 0.0)
            torch.cuda.synchronize()
            assert torch.equal(P3, P4) and torch.equal(U3, U0) and torch.equal(U4, U0)


def test_noalloc_md_update_rejects_too_large_a_lattice():
    import torch
    from paper_1611_00298_amd import Context
    from paper_1611_00298_amd._lib import EOFA_EINVAL, EOFAError
    L = (24, 24, 24, 80)   # 1105920 sites > 1048576
    assert L[0] * L[1] * L[2] * L[3] > MAX_SITES
    U0 = _identity_links(L)
    P0 = torch.zeros_like(U0)
    kin = torch.zeros((1,), dtype=torch.float64, device="cuda")
    with Context(L, 4, U0) as ctx:
        U, P = U0.clone(), P0.clone()
        with pytest.raises(EOFAError) as e:
            ctx.md_update_noalloc(U, P, None, 0.0, 0.1, kinetic=kin)
        assert e.value.code == EOFA_EINVAL and "too large" in str(e.value)
        torch.cuda.synchronize()
        assert torch.equal(U, U0) and kin.item() == 0.0   # nothing ran
