"""Pins of the oracle's Dirac operator against facts fixed by the definition and mathematics.

Each test is chosen so that a plausible slip in oracle/dslash.py (a dropped term,
a wrong sign, a wrong link site, a transposed instead of daggered link, a wrong
phase or boundary sign) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import dense, free, geometry
from oracle.dslash import (NAIK_COEFF, apply_m, colour_rotate, dslash_at_sites, dslash_eo,
                           dslash_full, gauge_transform_links, pure_gauge_links)
from stag_inputs import fat_field, gaussian_full_field, gaussian_source, random_gauge_transform, random_su3_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def links(dims, seed=7):
    return fat_field(dims, seed), random_su3_field(dims, seed + 1)


def inner(a, b):
    return np.vdot(a, b)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (8, 10, 8, 8)])
def test_delta_locality_and_values(dims):
    """D on a unit vector at y is nonzero only at y +- mu, y +- 3mu, with the folded link columns there."""
    fat, lng = links(dims)
    Lx, Ly, Lz, Lt = dims
    y = (3, 4, 2, Lt - 1)          # t = Lt-1: forward time hops from y wrap
    c = 1
    chi = np.zeros((Lt, Lz, Ly, Lx, 3), dtype=np.complex128)
    chi[y[3], y[2], y[1], y[0], c] = 1.0
    out = dslash_full(fat, lng, chi, dims, True, NAIK_COEFF)
    expected = np.zeros_like(out)
    for mu in range(4):
        for k, U, cf in ((1, fat, 1.0), (3, lng, NAIK_COEFF)):
            # output site n = y - k mu: forward term eta(n) s(n,k) U(n)[:, c]
            n = list(y)
            n[mu] = (y[mu] - k) % dims[mu]
            eta_n = (-1.0) ** (sum(n[:mu]) % 2)
            wraps = (n[mu] + k) // dims[mu]
            s = (-1.0) ** wraps if mu == 3 else 1.0
            expected[n[3], n[2], n[1], n[0]] += cf * eta_n * s * U[mu, n[3], n[2], n[1], n[0]][:, c]
            # output site n = y + k mu: backward term -eta(n) s(y,k) U(y)^dag[:, c]
            n = list(y)
            n[mu] = (y[mu] + k) % dims[mu]
            eta_n = (-1.0) ** (sum(n[:mu]) % 2)
            wraps = (y[mu] + k) // dims[mu]
            s = (-1.0) ** wraps if mu == 3 else 1.0
            expected[n[3], n[2], n[1], n[0]] -= cf * eta_n * s * U[mu, y[3], y[2], y[1], y[0]].conj().T[:, c]
    np.testing.assert_allclose(out, expected, atol=1e-15)
    assert np.count_nonzero(np.abs(out).sum(-1) > 0) == 16


@pytest.mark.parametrize("dims", [(4, 4, 6, 8), (2, 4, 6, 2), (6, 2, 4, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("antiperiodic", [True, False])
def test_anti_hermitian(dims, antiperiodic):
    """<psi, D chi> = -<D psi, chi> for any links, unitary or not (also when hops wrap several times)."""
    fat, lng = links(dims, 11)
    psi = gaussian_full_field(dims, 1)
    chi = gaussian_full_field(dims, 2)
    lhs = inner(psi, dslash_full(fat, lng, chi, dims, antiperiodic))
    rhs = -inner(dslash_full(fat, lng, psi, dims, antiperiodic), chi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_eo_blocks_are_negative_adjoints():
    """D_eo = -D_oe^dag, and D maps each parity to the other."""
    dims = (4, 6, 4, 8)
    fat, lng = links(dims, 3)
    a = gaussian_source(dims, 5)[0]
    b = gaussian_source(dims, 6)[0]
    lhs = inner(a, dslash_eo(fat, lng, b, dims, 0))
    rhs = -inner(dslash_eo(fat, lng, a, dims, 1), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    full = geometry.embed(b, dims, 1)
    out = dslash_full(fat, lng, full, dims)
    assert np.abs(geometry.restrict(out, dims, 1)).max() == 0.0


@pytest.mark.parametrize("naik", [NAIK_COEFF, 0.0])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (4, 6, 8, 10), (2, 4, 6, 2)])
def test_free_field_plane_waves(dims, naik):
    """Unit links: even-site plane waves are eigenvectors of -D_eo D_oe with 4 sum (sin p + c_N sin 3p)^2."""
    U = free.unit_links(dims)
    rng = np.random.default_rng(0)
    pgrid = free.momenta(dims, True)
    for _ in range(6):
        p = [g[rng.integers(len(g))] for g in pgrid]
        wave = free.plane_wave(dims, p)[..., None] * np.array([0.3, -1.0j, 0.7])
        v = geometry.restrict(wave, dims, 0)
        t = dslash_eo(U, U, v, dims, 1, True, naik)
        mv = -dslash_eo(U, U, t, dims, 0, True, naik)
        lam = free.free_eigenvalue(p, naik)
        np.testing.assert_allclose(mv, lam * v, atol=1e-12 * max(1.0, lam))


def test_free_field_one_hop_is_sum_of_sin_squared():
    """The one-hop case: with Eq. (5) (no 1/2), -D^2 has eigenvalues 4 sum_mu sin^2 p_mu."""
    p = (0.3, 1.1, 2.0, 0.7)
    assert free.free_eigenvalue(p, 0.0) == pytest.approx(4 * sum(np.sin(q) ** 2 for q in p), rel=1e-15)


def test_gauge_covariance():
    """D[U^g](g chi) = g D[U] chi with U^g_mu(n) = g(n) U_mu(n) g(n + k mu)^dag, also for non-unitary links."""
    dims = (4, 6, 8, 8)
    fat, lng = links(dims, 21)
    g = random_gauge_transform(dims, 22)
    chi = gaussian_full_field(dims, 23)
    fat_g, lng_g = gauge_transform_links(fat, lng, g, dims)
    lhs = dslash_full(fat_g, lng_g, colour_rotate(g, chi), dims)
    rhs = colour_rotate(g, dslash_full(fat, lng, chi, dims))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_dense_builder_matches_vectorised():
    """The scalar-loop dense matrix and the vectorised operator agree, and the matrix is anti-Hermitian."""
    for dims in [(2, 2, 2, 2), (2, 4, 2, 4), (4, 2, 2, 8)]:
        fat, lng = links(dims, 31)
        D = dense.dense_dslash(fat, lng, dims)
        chi = gaussian_full_field(dims, 32)
        out = dslash_full(fat, lng, chi, dims)
        np.testing.assert_allclose(D @ chi.reshape(-1), out.reshape(-1), atol=1e-13)
        np.testing.assert_allclose(D, -D.conj().T, atol=1e-15)


def test_dslash_at_sites_matches_full():
    dims = (6, 4, 8, 8)
    fat, lng = links(dims, 41)
    v = gaussian_source(dims, 42)[0]
    for par in (0, 1):
        ref = dslash_eo(fat, lng, v, dims, par)
        half = len(v)
        cbs = np.arange(half)
        np.testing.assert_allclose(dslash_at_sites(fat, lng, v, dims, par, cbs), ref, atol=1e-13)


def test_normal_operator_hermitian_positive():
    """<psi, M psi> = 4 m^2 ||psi||^2 + ||D_oe psi||^2 and M is Hermitian."""
    dims = (4, 4, 6, 8)
    fat, lng = links(dims, 51)
    m = 0.05
    a = gaussian_source(dims, 52)[0]
    b = gaussian_source(dims, 53)[0]
    ma = apply_m(fat, lng, a, dims, m)
    quad = inner(a, ma)
    t = dslash_eo(fat, lng, a, dims, 1)
    assert abs(quad.imag) <= 1e-13 * abs(quad)
    assert quad.real == pytest.approx(4 * m * m * inner(a, a).real + inner(t, t).real, rel=1e-13)
    lhs = inner(b, ma)
    rhs = inner(apply_m(fat, lng, b, dims, m), a)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_pure_gauge_solve_has_known_answer():
    """Pure gauge links give M[U] = G M[1] G^dag, so x = G x_free(G^dag b)."""
    dims = (4, 4, 4, 8)
    g = random_gauge_transform(dims, 61)
    fat, lng = pure_gauge_links(g, dims)
    b = gaussian_source(dims, 62)[0]
    m = 0.1
    ge = g.reshape(-1, 3, 3)[geometry.parity(dims).reshape(-1) == 0]
    gdag_b = np.einsum("nba,nb->na", ge.conj(), b)
    x = np.einsum("nab,nb->na", ge, free.free_solve(gdag_b, dims, m))
    np.testing.assert_allclose(apply_m(fat, lng, x, dims, m), b, atol=1e-11)


def test_fft_free_solve_inverts_operator():
    dims = (8, 8, 8, 8)
    U = free.unit_links(dims)
    b = gaussian_source(dims, 71)[0]
    x = free.free_solve(b, dims, 0.05)
    np.testing.assert_allclose(apply_m(U, U, x, dims, 0.05), b, atol=1e-11)


def test_two_to_the_four_free_operator_is_diagonal():
    g = json.load(open(os.path.join(GOLDEN, "free_2x2x2x2.json")))
    dims = tuple(g["dims"])
    U = free.unit_links(dims)
    M = dense.dense_normal_operator(U, U, dims, g["mass"], True, g["naik"])
    np.testing.assert_allclose(M, g["m_diagonal"] * np.eye(M.shape[0]), atol=1e-14)


@pytest.mark.parametrize("dims", [(4, 4, 6, 8), (2, 4, 2, 2), (6, 2, 4, 6)])
def test_site_matrices_reproduce_operator(dims):
    """The 16 per-site matrices (storage order of the low-precision path) reproduce D_{p,1-p} exactly."""
    from oracle.lowprec import apply_site_matrices, site_matrices

    fat, lng = links(dims, 81)
    v = gaussian_source(dims, 82)[0]
    for par in (0, 1):
        mats, nbr = site_matrices(fat, lng, dims, par)
        np.testing.assert_allclose(apply_site_matrices(mats, nbr, v), dslash_eo(fat, lng, v, dims, par), atol=1e-13)


def test_su3_third_row_is_conjugate_cross_product():
    """Paper Sec. 3.3, Eq. SU3rec: for U in SU(3), row 3 = (row 1 x row 2)^*."""
    U = random_su3_field((4, 4, 4, 4), 91).reshape(-1, 3, 3)
    np.testing.assert_allclose(U[:, 2], np.conj(np.cross(U[:, 0], U[:, 1])), atol=1e-14)
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 6, 8), (2, 4, 2, 2), (4, 2, 4, 6)])
def test_twelve_parameter_long_links_rebuild_the_operator(dims):
    """Rebuilding the three-hop matrices from two rows and the folded scalars leaves D unchanged."""
    from oracle.lowprec import K_LONG, apply_site_matrices, folded_scalars, rebuild_third_rows, site_matrices

    fat, lng = links(dims, 92)
    v = gaussian_source(dims, 93)[0]
    for par in (0, 1):
        mats, nbr = site_matrices(fat, lng, dims, par)
        sc = folded_scalars(dims, par)
        # the scalars are what the matrices carry: mats = s * (an SU(3) matrix) for three-hop k
        for k in K_LONG:
            np.testing.assert_allclose(np.abs(np.linalg.det(mats[:, k])), np.abs(sc[:, k]) ** 3, rtol=1e-12)
        reb = rebuild_third_rows(mats, sc, K_LONG)
        np.testing.assert_allclose(reb, mats, atol=1e-15)
        np.testing.assert_allclose(apply_site_matrices(reb, nbr, v), dslash_eo(fat, lng, v, dims, par), atol=1e-13)


@pytest.mark.parametrize("dims", [(4, 4, 6, 8), (6, 2, 4, 6)])
def test_site_matrices_at_chosen_sites(dims):
    """site_matrices / folded_scalars for chosen checkerboard indices are the rows of the whole-lattice
    ones, and applied to a vector they give the site-by-site operator dslash_at_sites."""
    from oracle.lowprec import apply_site_matrices, folded_scalars, output_sites, site_matrices

    fat, lng = links(dims, 94)
    v = gaussian_source(dims, 95)[0]
    half = int(np.prod(dims)) // 2
    cbs = np.array([0, half - 1, 5, 3, 5, half // 2 + 1])
    for par in (0, 1):
        np.testing.assert_array_equal(output_sites(dims, par, np.arange(half)), output_sites(dims, par))
        mats, nbr = site_matrices(fat, lng, dims, par)
        m_s, n_s = site_matrices(fat, lng, dims, par, cbs=cbs)
        np.testing.assert_array_equal(m_s, mats[cbs])
        np.testing.assert_array_equal(n_s, nbr[cbs])
        np.testing.assert_array_equal(folded_scalars(dims, par, cbs=cbs), folded_scalars(dims, par)[cbs])
        np.testing.assert_allclose(apply_site_matrices(m_s, n_s, v), dslash_at_sites(fat, lng, v, dims, par, cbs),
                                   atol=1e-13)


def test_chunked_operator_matches_whole_lattice_operator():
    """The chunked, threaded M (several right-hand sides, one mass each, ragged last chunk) equals apply_m."""
    from oracle.cg import true_residual, true_residuals
    from oracle.dslash import apply_m_chunked

    dims = (6, 4, 4, 6)
    fat, lng = links(dims, 41)
    b = gaussian_source(dims, 42, 3)
    masses = [0.05, 0.1, 0.3]
    for chunk, workers in ((7, 1), (50, 3), (1 << 16, 2)):
        got = apply_m_chunked(fat, lng, b, dims, masses, chunk=chunk, workers=workers)
        for r in range(3):
            np.testing.assert_allclose(got[r], apply_m(fat, lng, b[r], dims, masses[r]), atol=1e-13)
    one = apply_m_chunked(fat, lng, b[1], dims, 0.1, chunk=11)
    np.testing.assert_allclose(one, apply_m(fat, lng, b[1], dims, 0.1), atol=1e-13)
    x = gaussian_source(dims, 43, 3)
    rs = true_residuals(lambda v: apply_m_chunked(fat, lng, v, dims, masses, chunk=64), b, x)
    for r in range(3):
        assert rs[r] == pytest.approx(true_residual(lambda v: apply_m(fat, lng, v, dims, masses[r]), b[r], x[r]),
                                      rel=1e-12)
