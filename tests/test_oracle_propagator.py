"""Pins of the oracle's point-source propagator and pion correlator (oracle/propagator.py) against facts
fixed by the definition: the dense inverse of the full operator M = 2m + D, the Dirac equation M G = delta
itself, the sum rule sum_t C(t) = sum_c chi^(c)(x0)_c, and the correlator summed site by site."""
import numpy as np
import pytest

from oracle import dense, geometry
from oracle.dslash import NAIK_COEFF, dslash_full
from oracle.propagator import correlator, even_solutions, full_field, point_sources, propagator
from stag_inputs import fat_field, random_su3_field


def links(dims, seed):
    return fat_field(dims, seed), random_su3_field(dims, seed + 1)


def test_matches_the_dense_inverse_of_the_full_operator():
    """G = (2m + D)^{-1} delta from a dense solve with the scalar-loop matrix (written apart from the
    vectorised operator) equals the propagator built from the even-site solve."""
    dims = (2, 4, 2, 4)
    fat, lng = links(dims, 301)
    m = 0.3
    sites = [(0, 0, 0, 0), (1, 1, 0, 2)]
    b = point_sources(dims, sites)
    chi = even_solutions(fat, lng, dims, m, b, tol=1e-14)
    g_e, g_o = propagator(fat, lng, dims, m, chi)
    M = 2.0 * m * np.eye(3 * np.prod(dims)) + dense.dense_dslash(fat, lng, dims)
    Lx, Ly, Lz, Lt = dims
    for s, (x, y, z, t) in enumerate(sites):
        for c in range(3):
            rhs = np.zeros(3 * np.prod(dims), dtype=np.complex128)
            rhs[3 * (x + Lx * (y + Ly * (z + Lz * t))) + c] = 1.0
            ref = np.linalg.solve(M, rhs)
            got = full_field(g_e[3 * s + c], g_o[3 * s + c], dims).reshape(-1)
            np.testing.assert_allclose(got, ref, atol=1e-11)


@pytest.mark.parametrize("naik", [NAIK_COEFF, 0.0])
def test_solves_the_dirac_equation(naik):
    dims = (4, 4, 4, 8)
    fat, lng = links(dims, 311)
    m = 0.1
    b = point_sources(dims, [(2, 1, 3, 4)])
    chi = even_solutions(fat, lng, dims, m, b, tol=1e-12, naik=naik)
    g_e, g_o = propagator(fat, lng, dims, m, chi, naik=naik)
    for c in range(3):
        G = full_field(g_e[c], g_o[c], dims)
        MG = 2.0 * m * G + dslash_full(fat, lng, G, dims, naik=naik)
        delta = full_field(b[c], np.zeros_like(b[c]), dims)
        assert np.linalg.norm(MG - delta) <= 1e-10


def test_correlator_sum_rule():
    """sum_t C(t) = sum_c chi^(c)(x0)_c, because M M^dag is the normal operator."""
    dims = (4, 4, 4, 8)
    fat, lng = links(dims, 321)
    m = 0.1
    sites = [(0, 0, 0, 0), (1, 2, 3, 2)]
    b = point_sources(dims, sites)
    chi = even_solutions(fat, lng, dims, m, b, tol=1e-13)
    C = correlator(*propagator(fat, lng, dims, m, chi), dims)
    for s, (x, y, z, t) in enumerate(sites):
        cb = geometry.cb_of_site(x, y, z, t, dims)
        diag = sum(chi[3 * s + c, cb, c] for c in range(3))
        assert abs(diag.imag) <= 1e-10 * abs(diag)
        assert C[s].sum() == pytest.approx(diag.real, rel=1e-10)
        assert np.all(C[s] > 0)


def test_correlator_summed_site_by_site():
    dims = (2, 2, 4, 6)
    rng = np.random.default_rng(5)
    half = np.prod(dims) // 2
    g_e = rng.normal(size=(6, half, 3)) + 1j * rng.normal(size=(6, half, 3))
    g_o = rng.normal(size=(6, half, 3)) + 1j * rng.normal(size=(6, half, 3))
    C = correlator(g_e, g_o, dims)
    ref = np.zeros((2, dims[3]))
    for s in range(2):
        for c in range(3):
            for par, g in ((0, g_e), (1, g_o)):
                for cb in range(half):
                    t = geometry.site_of_cb(cb, par, dims)[3]
                    ref[s, t] += np.sum(np.abs(g[3 * s + c, cb]) ** 2)
    np.testing.assert_allclose(C, ref, rtol=1e-13)


def test_point_sources():
    dims = (4, 4, 4, 4)
    b = point_sources(dims, [(1, 1, 0, 0)])
    assert b.shape == (3, 128, 3) and b.sum() == 3
    cb = geometry.cb_of_site(1, 1, 0, 0, dims)
    assert all(b[c, cb, c] == 1 for c in range(3))
    with pytest.raises(ValueError):
        point_sources(dims, [(1, 0, 0, 0)])
