"""The index scheme of the block-sharing hop, checked on the CPU against the
lattice conventions of the oracle (natural site order, parity (x+y+z+t) mod 2,
periodic neighbours).

The hop's workgroups hold whole 2x2x2x2 blocks at even coordinates.  A block's
8 sites of the output parity p sit in slots j = b_y + 2 b_z + 4 b_t (b the
offsets in the block) and then b_x = (b_y + b_z + b_t + p) mod 2.  Each
work-item loads the block's opposite-parity site with the same (y, z, t), its
inside neighbour along x, and shares it; the inside neighbours along y, z and
t are those loaded by slots j^1, j^2 and j^4, and along every direction
exactly one of the two neighbours lies inside the block (+mu if b_mu = 0).
The GPU parity tests check the kernels; this pins the scheme they rely on.
Also the checkerboard index of a site (natural index // 2) does not depend
on b_x, so one block table serves both parities."""
import itertools

import pytest

import oracle

SHAPES = [(4, 4, 4, 4), (2, 2, 4, 4), (4, 4, 2, 2), (2, 2, 2, 6), (6, 2, 4, 2), (8, 4, 4, 8)]


def natural(L, c):
    x, y, z, t = c
    return x + L[0] * (y + L[1] * (z + L[2] * t))


def shift(L, c, mu, step):
    e = list(c)
    e[mu] = (e[mu] + step) % L[mu]
    return tuple(e)


def parity_of(mask, c):
    x, y, z, t = c
    return int(mask[t, z, y, x])


@pytest.mark.parametrize("L", SHAPES, ids=lambda L: "x".join(map(str, L)))
def test_block_slots_and_shared_neighbours(L):
    mask = oracle.Lattice(L, 2).parity_mask()
    for p in (0, 1):
        for B in itertools.product(*(range(n // 2) for n in L)):
            origin = tuple(2 * v for v in B)
            sites = {}
            for j in range(8):
                by, bz, bt = j & 1, (j >> 1) & 1, j >> 2
                bx = (by + bz + bt + p) % 2
                c = (origin[0] + bx, origin[1] + by, origin[2] + bz, origin[3] + bt)
                assert parity_of(mask, c) == p
                sites[j] = (c, (bx, by, bz, bt))
            # the 8 slots are the block's 8 sites of parity p, each once
            assert len({natural(L, c) for c, _ in sites.values()}) == 8
            # the x-inside partner of slot j: same (y, z, t), opposite parity
            partner = {}
            for j, (c, b) in sites.items():
                step = 1 if b[0] == 0 else -1
                q = shift(L, c, 0, step)
                assert q[1:] == c[1:] and parity_of(mask, q) == 1 - p
                assert all(origin[m] <= q[m] < origin[m] + 2 for m in range(4))
                partner[j] = q
            for j, (c, b) in sites.items():
                for mu in range(4):
                    inside = shift(L, c, mu, 1 if b[mu] == 0 else -1)
                    outside = shift(L, c, mu, -1 if b[mu] == 0 else 1)
                    # the inside neighbour lies in the block (for extent 2 the
                    # two neighbours coincide, and the scheme still names it)
                    assert all(origin[m] <= inside[m] < origin[m] + 2 for m in range(4))
                    if L[mu] > 2:
                        assert not all(origin[m] <= outside[m] < origin[m] + 2 for m in range(4))
                    if mu == 0:
                        assert inside == partner[j]
                    else:
                        assert inside == partner[j ^ (1 << (mu - 1))]
            # the checkerboard index does not depend on b_x: the block table is
            # the same for both parities
            for j, (c, b) in sites.items():
                other = (c[0] ^ 1,) + c[1:]
                assert natural(L, c) // 2 == natural(L, other) // 2


def test_block_scheme_detects_a_wrong_slot_order():
    """A mistake the scheme must not tolerate: with slots ordered
    j = b_z + 2 b_y + 4 b_t (y and z swapped), the inside neighbour along y
    is no longer the partner of slot j^1."""
    L = (4, 4, 4, 4)
    p = 0
    origin = (0, 0, 0, 0)
    bad = False
    for j in range(8):
        bz, by, bt = j & 1, (j >> 1) & 1, j >> 2
        bx = (by + bz + bt + p) % 2
        c = (bx, by, bz, bt)
        inside_y = shift(L, c, 1, 1 if by == 0 else -1)
        k = j ^ 1
        kz, ky, kt = k & 1, (k >> 1) & 1, k >> 2
        kx = (ky + kz + kt + p) % 2
        partner_k = ((kx ^ 1), ky, kz, kt)
        bad |= inside_y != tuple(origin[m] + partner_k[m] for m in range(4))
    assert bad
