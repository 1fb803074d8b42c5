"""The seeded input generators (dwf_inputs): SU(3) links, Hermitian
traceless momenta, Gaussian spinors; same seed, same field."""
import numpy as np

import dwf_inputs as din


def test_random_links_are_su3():
    U = din.random_gauge((4, 2, 4, 2), 0.8, 7)
    UU = U @ np.swapaxes(U.conj(), -1, -2)
    assert np.abs(UU - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    assert U.shape == (4, 2, 4, 2, 4, 3, 3)   # (mu, t, z, y, x, a, b)


def test_link_spread_follows_eps():
    """exp(i eps H): eps -> 0 gives the unit field; larger eps, rougher links."""
    d = [np.abs(din.random_gauge((2, 2, 2, 2), e, 8) - np.eye(3)).mean() for e in (1e-6, 0.1, 0.5)]
    assert d[0] < 1e-5 and d[0] < d[1] < d[2]


def test_momenta_hermitian_traceless_unit_normal():
    P = din.gaussian_momenta((4, 4, 4, 4), 9)
    assert np.abs(P - np.swapaxes(P.conj(), -1, -2)).max() < 1e-15
    assert np.abs(np.trace(P, axis1=-2, axis2=-1)).max() < 1e-14
    # P = sum_a p^a lambda^a / 2 with p^a ~ N(0, 1): tr P^2 = (1/2) sum_a (p^a)^2, mean 4 per link
    kin = (P * np.swapaxes(P, -1, -2)).sum(axis=(-2, -1)).real
    assert abs(kin.mean() - 4.0) < 0.1


def test_gaussian_spinors():
    e = din.gaussian_4d((8, 8, 8, 8), 10)
    assert e.shape == (8, 8, 8, 8, 4, 3)
    assert abs(e.real.var() - 0.5) < 0.01 and abs(e.imag.var() - 0.5) < 0.01
    assert abs(e.mean()) < 0.01
    p = din.gaussian_5d((4, 4, 4, 4), 3, 11)
    assert p.shape == (3, 4, 4, 4, 4, 4, 3)


def test_same_seed_same_field():
    a = din.random_gauge((2, 2, 2, 4), 0.5, 12)
    b = din.random_gauge((2, 2, 2, 4), 0.5, 12)
    c = din.random_gauge((2, 2, 2, 4), 0.5, 13)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(din.gaussian_4d((2, 2, 2, 2), 5), din.gaussian_4d((2, 2, 2, 2), 5))
