"""Pins of the link-fattening oracle (oracle/fatten.py) against facts its definition fixes.

A slip in the path table (a missing or duplicated path, a wrong displacement, a wrong coefficient or
tadpole power) fails the unit-link normalisation or the transverse-identity stencil; a link taken at
the wrong site or without its dagger on a backward step fails gauge covariance; a wrong three-hop product
fails its closed form.
"""
import itertools

import numpy as np
import pytest

from oracle import fatten, free, geometry
from oracle.dslash import dslash_eo
from stag_inputs import random_gauge_transform, random_su3_field


def unit(dims):
    return free.unit_links(dims)


def test_path_table_counts_and_endpoints():
    for mu in range(4):
        ps = fatten.paths(mu)
        counts = {}
        for cls, steps in ps:
            counts[cls] = counts.get(cls, 0) + 1
            end = [0, 0, 0, 0]
            for nu, s in steps:
                end[nu] += s
            assert end == [1 if d == mu else 0 for d in range(4)]
            assert sum(1 for nu, s in steps if nu == mu) == 1     # exactly one step along mu
        assert counts == {"one": 1, "three": 6, "five": 24, "seven": 48, "lepage": 6}


@pytest.mark.parametrize("u0", [1.0, 0.87])
def test_unit_links_give_the_tree_level_normalisation(u0):
    """Unit links: every path product is 1, so V = sum of (count x coefficient) = 9/8 at u0 = 1."""
    dims = (4, 4, 4, 6)
    V = fatten.fat_links(unit(dims), dims, u0)
    expect = 5 / 8 + 6 / 16 / u0 ** 2 + 24 / 64 / u0 ** 4 + 48 / 384 / u0 ** 6 - 6 / 16 / u0 ** 4
    if u0 == 1.0:
        assert expect == pytest.approx(9 / 8, abs=1e-15)
    np.testing.assert_allclose(V, expect * unit(dims), atol=1e-14)
    np.testing.assert_allclose(fatten.long_links(unit(dims), dims), unit(dims), atol=1e-15)


def _stencil_weight(d, u0=1.0):
    """Weight of the mu-link displaced by the transverse vector d when every transverse link is 1.

    A staple through transverse steps multiplies to 1 on its transverse legs, so its product is the mu
    link at the displaced site: one three-link staple per +-nu, two five-link staples (two orders of
    nu, rho) per diagonal displacement, six seven-link staples (orders of nu, rho, sigma) per cube
    corner, one Lepage path per +-2 nu."""
    nz = [abs(v) for v in d if v != 0]
    if not nz:
        return 5 / 8
    if nz == [1]:
        return 1 / 16 / u0 ** 2
    if nz == [2]:
        return -1 / 16 / u0 ** 4
    if nz == [1, 1]:
        return 2 / 64 / u0 ** 4
    if nz == [1, 1, 1]:
        return 6 / 384 / u0 ** 6
    return 0.0


@pytest.mark.parametrize("mu,dims", [(3, (6, 6, 6, 4)), (0, (4, 6, 6, 6)), (1, (6, 4, 6, 6))])
def test_transverse_identity_reduces_to_a_stencil(mu, dims):
    """With U_nu = 1 for nu != mu and U_mu random SU(3), V_mu(n) = sum_d w(d) U_mu(n + d) exactly."""
    U = unit(dims)
    U[mu] = random_su3_field(dims, 11)[mu]
    V = fatten.fat_links(U, dims)
    trans = [d for d in range(4) if d != mu]
    expect = np.zeros_like(U[mu])
    for disp in itertools.product(range(-2, 3), repeat=3):
        w = _stencil_weight(disp)
        if w == 0.0:
            continue
        off = [0, 0, 0, 0]
        for d, v in zip(trans, disp):
            off[d] = v
        expect += w * np.roll(U[mu], shift=(-off[3], -off[2], -off[1], -off[0]), axis=(0, 1, 2, 3))
    np.testing.assert_allclose(V[mu], expect, atol=1e-14)


def test_long_link_of_commuting_links_adds_the_angles():
    """U_mu(n) = exp(i theta(n) H) with one Hermitian H: W_mu(n) = exp(i (theta(n) + theta(n+mu) + theta(n+2mu)) H)."""
    dims = (4, 6, 4, 6)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    H = A + A.conj().T
    w, Q = np.linalg.eigh(H)
    U = unit(dims)
    thetas = []
    for mu in range(4):
        th = rng.uniform(-np.pi, np.pi, size=(dims[3], dims[2], dims[1], dims[0]))
        thetas.append(th)
        U[mu] = np.einsum("ij,...j,kj->...ik", Q, np.exp(1j * th[..., None] * w), Q.conj())
    W = fatten.long_links(U, dims)
    for mu in range(4):
        tot = sum(geometry.shift(thetas[mu], mu, k) for k in range(3))
        expect = np.einsum("ij,...j,kj->...ik", Q, np.exp(1j * tot[..., None] * w), Q.conj())
        np.testing.assert_allclose(W[mu], expect, atol=1e-12)


@pytest.mark.parametrize("u0", [1.0, 0.9])
def test_gauge_covariance(u0):
    """U_mu(n) -> g(n) U_mu(n) g(n+mu)^dag gives V -> g V g(n+mu)^dag and W -> g W g(n+3mu)^dag."""
    dims = (4, 4, 6, 4)
    U = random_su3_field(dims, 21)
    g = random_gauge_transform(dims, 22)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = np.einsum("...ab,...bc,...dc->...ad", g, U[mu], geometry.shift(g, mu, 1).conj())
    V, W = fatten.fat_links(U, dims, u0), fatten.long_links(U, dims)
    Vg, Wg = fatten.fat_links(Ug, dims, u0), fatten.long_links(Ug, dims)
    for mu in range(4):
        np.testing.assert_allclose(
            Vg[mu], np.einsum("...ab,...bc,...dc->...ad", g, V[mu], geometry.shift(g, mu, 1).conj()), atol=1e-13)
        np.testing.assert_allclose(
            Wg[mu], np.einsum("...ab,...bc,...dc->...ad", g, W[mu], geometry.shift(g, mu, 3).conj()), atol=1e-13)


def test_one_site_walk_matches_the_field_version():
    dims = (4, 6, 4, 4)
    U = random_su3_field(dims, 31)
    V, W = fatten.fat_links(U, dims, 0.95), fatten.long_links(U, dims)
    rng = np.random.default_rng(5)
    for _ in range(6):
        x, y, z, t = (int(rng.integers(L)) for L in dims)
        mu = int(rng.integers(4))
        np.testing.assert_allclose(fatten.fat_link_at(U, dims, (x, y, z, t), mu, 0.95), V[mu, t, z, y, x],
                                   atol=1e-14)
        np.testing.assert_allclose(fatten.long_link_at(U, dims, (x, y, z, t), mu), W[mu, t, z, y, x], atol=1e-15)


def test_fattened_free_field_has_the_improved_dispersion():
    """Fattened unit links in the operator (c_N = -1/24): -D^2 = 4 sum (9/8 sin p - 1/24 sin 3p)^2."""
    dims = (4, 4, 6, 8)
    U = unit(dims)
    V, W = fatten.fat_links(U, dims), fatten.long_links(U, dims)
    rng = np.random.default_rng(9)
    pg = free.momenta(dims, True)
    for _ in range(4):
        p = [g[rng.integers(len(g))] for g in pg]
        v = geometry.restrict(free.plane_wave(dims, p)[..., None] * np.array([1.0, 0.5j, -0.2]), dims, 0)
        mv = -dslash_eo(V, W, dslash_eo(V, W, v, dims, 1), dims, 0)
        lam = 4 * sum((9 / 8 * np.sin(q) - np.sin(3 * q) / 24) ** 2 for q in p)
        np.testing.assert_allclose(mv, lam * v, atol=1e-12 * max(1.0, lam))
