"""Pins of the oracle's CG (paper Fig. 1) against direct solves and closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import dense, free
from oracle.cg import cg, true_residual
from oracle.dslash import apply_m
from stag_inputs import fat_field, gaussian_source, random_su3_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_cg_matches_dense_direct_solve(dims):
    """Random non-unitary fat + SU(3) long links: CG's x agrees with numpy.linalg.solve within kappa * tol."""
    fat, lng = fat_field(dims, 3), random_su3_field(dims, 4)
    m = 0.05
    b = gaussian_source(dims, 5)[0]
    M = dense.dense_normal_operator(fat, lng, dims, m)
    x_ref = np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)
    res = cg(lambda v: apply_m(fat, lng, v, dims, m), b, tol=1e-10)
    assert res.converged and res.true_resid <= 1e-10
    ev = np.linalg.eigvalsh(M)
    kappa = ev[-1] / ev[0]
    err = np.linalg.norm(res.x - x_ref) / np.linalg.norm(x_ref)
    assert err <= kappa * 1e-10
    # M as a callable and as a dense matrix are the same map
    np.testing.assert_allclose(M @ b.reshape(-1), apply_m(fat, lng, b, dims, m).reshape(-1), atol=1e-12)


def test_free_2x2x2x2_converges_in_one_iteration():
    g = json.load(open(os.path.join(GOLDEN, "free_2x2x2x2.json")))
    dims = tuple(g["dims"])
    U = free.unit_links(dims)
    b = gaussian_source(dims, 9)[0]
    res = cg(lambda v: apply_m(U, U, v, dims, g["mass"]), b, tol=1e-10, record=2)
    assert res.iters == 1
    assert res.alphas[0] == pytest.approx(1.0 / g["m_diagonal"], rel=1e-14)


def test_free_field_cg_iterations_bounded_by_distinct_eigenvalues():
    """In exact arithmetic CG needs at most K iterations, K = number of distinct eigenvalues."""
    dims = (4, 4, 4, 4)
    U = free.unit_links(dims)
    m = 0.2
    lam = free.free_spectrum(dims)
    K = len(np.unique(np.round(lam, 10)))
    b = gaussian_source(dims, 10)[0]
    res = cg(lambda v: apply_m(U, U, v, dims, m), b, tol=1e-10)
    assert res.converged and res.iters <= K
    np.testing.assert_allclose(res.x, free.free_solve(b, dims, m), rtol=0, atol=1e-9)


def test_cg_free_field_8x8x8x8_matches_fft():
    dims = (8, 8, 8, 8)
    U = free.unit_links(dims)
    m = 0.05
    b = gaussian_source(dims, 11)[0]
    res = cg(lambda v: apply_m(U, U, v, dims, m), b, tol=1e-10)
    x = free.free_solve(b, dims, m)
    assert res.true_resid <= 1e-10
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) <= 1e-10 / (4 * m * m) * 20


def test_cg_restart_and_warm_start():
    """A warm start at the solution needs zero iterations; a bad tolerance path restarts from x."""
    dims = (4, 4, 4, 4)
    fat, lng = fat_field(dims, 12), random_su3_field(dims, 13)
    m = 0.1
    A = lambda v: apply_m(fat, lng, v, dims, m)
    b = gaussian_source(dims, 14)[0]
    res = cg(A, b, tol=1e-10)
    res2 = cg(A, b, tol=1e-10, x0=res.x)
    assert res2.iters == 0 and res2.converged
    assert true_residual(A, b, res.x) <= 1e-10


def test_cg_zero_source():
    dims = (2, 2, 2, 2)
    U = free.unit_links(dims)
    res = cg(lambda v: apply_m(U, U, v, dims, 0.1), np.zeros((8, 3), complex))
    assert res.converged and res.iters == 0 and not res.x.any()
