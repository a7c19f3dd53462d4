"""Pins of the network oracle (covariance, linearity, adjoints, finite-difference gradients) and of FCG."""
import numpy as np
import pytest

from oracle import dense, geometry
from oracle.cg import cg
from oracle.dslash import apply_m, colour_rotate, gauge_transform_links
from oracle.fcg import fcg
from oracle.net import (folded_fat, hermitian_weights, init_weights, layer_backward, layer_forward, loss_and_grads,
                        net_forward, transport, transport_adjoint)
from stag_inputs import fat_field, gaussian_full_field, gaussian_source, random_gauge_transform, random_su3_field

DIMS = (4, 4, 2, 6)


def test_transport_adjoints():
    """<phi, T_{+mu} psi> = <T_{-mu} phi, psi> for every direction."""
    fat = fat_field(DIMS, 1)
    Ft = folded_fat(fat, DIMS)
    psi = gaussian_full_field(DIMS, 2)
    phi = gaussian_full_field(DIMS, 3)
    for d in range(1, 9):
        lhs = np.vdot(phi, transport(Ft, psi, d))
        rhs = np.vdot(transport_adjoint(Ft, phi, d), psi)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_transports_sum_to_one_hop_operator():
    """sum_mu (T_{+mu} - T_{-mu}) is the one-hop Dirac operator of Eq. (5)."""
    from oracle.dslash import dslash_full

    fat = fat_field(DIMS, 4)
    Ft = folded_fat(fat, DIMS)
    psi = gaussian_full_field(DIMS, 5)
    acc = sum(transport(Ft, psi, 1 + mu) - transport(Ft, psi, 5 + mu) for mu in range(4))
    np.testing.assert_allclose(acc, dslash_full(fat, None, psi, DIMS), atol=1e-13)


def test_net_linear_and_gauge_covariant():
    fat = fat_field(DIMS, 6)
    W = init_weights([1, 3, 3, 1], 7, scale=1.0)
    r1 = gaussian_source(DIMS, 8)[0]
    r2 = gaussian_source(DIMS, 9)[0]
    Ft = folded_fat(fat, DIMS)
    out = net_forward(Ft, W, 0.3 * r1 - 2j * r2, DIMS)
    np.testing.assert_allclose(out, 0.3 * net_forward(Ft, W, r1, DIMS) - 2j * net_forward(Ft, W, r2, DIMS),
                               atol=1e-12)
    g = random_gauge_transform(DIMS, 10)
    fat_g, _ = gauge_transform_links(fat, None, g, DIMS)
    ge = g.reshape(-1, 3, 3)[geometry.parity(DIMS).reshape(-1) == 0]
    lhs = net_forward(folded_fat(fat_g, DIMS), W, np.einsum("nab,nb->na", ge, r1), DIMS)
    rhs = np.einsum("nab,nb->na", ge, net_forward(Ft, W, r1, DIMS))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_identity_network():
    fat = fat_field(DIMS, 11)
    W = [np.zeros((9, 1, 1), complex)]
    W[0][0, 0, 0] = 1.0
    r = gaussian_source(DIMS, 12)[0]
    np.testing.assert_allclose(net_forward(folded_fat(fat, DIMS), W, r, DIMS), r, atol=0)


def test_layer_backward_is_adjoint():
    fat = fat_field(DIMS, 13)
    Ft = folded_fat(fat, DIMS)
    W = init_weights([2, 3], 14, scale=1.0)[0]
    rng = np.random.default_rng(15)
    shp = (2,) + DIMS[::-1] + (3,)
    psi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    g = rng.standard_normal((3,) + shp[1:]) + 1j * rng.standard_normal((3,) + shp[1:])
    g_psi, _ = layer_backward(Ft, psi, W, g)
    assert abs(np.vdot(g, layer_forward(Ft, psi, W)) - np.vdot(g_psi, psi)) <= 1e-11 * abs(np.vdot(g_psi, psi))


def test_weight_gradients_match_finite_differences():
    fat = fat_field(DIMS, 16)
    Ft = folded_fat(fat, DIMS)
    W = init_weights([1, 2, 2, 1], 17, scale=1.0)
    pairs = [(gaussian_source(DIMS, 18 + i)[0], gaussian_source(DIMS, 30 + i)[0]) for i in range(2)]
    L0, grads = loss_and_grads(Ft, W, pairs, DIMS)
    rng = np.random.default_rng(19)
    h = 1e-6
    for _ in range(8):
        l = rng.integers(len(W))
        idx = tuple(rng.integers(s) for s in W[l].shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][idx] += h * unit
            Wm[l][idx] -= h * unit
            fd = (loss_and_grads(Ft, Wp, pairs, DIMS)[0] - loss_and_grads(Ft, Wm, pairs, DIMS)[0]) / (2 * h)
            an = 2 * (grads[l][idx].real if part == "re" else grads[l][idx].imag)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_residual_loss_gradients_match_finite_differences():
    from oracle.dslash import apply_m

    fat, lng = fat_field(DIMS, 40), random_su3_field(DIMS, 41)
    Ft = folded_fat(fat, DIMS)
    A = lambda v: apply_m(fat, lng, v, DIMS, 0.2)
    W = init_weights([1, 2, 1], 42, scale=1.0)
    pairs = [(gaussian_source(DIMS, 43)[0], None)]
    L0, grads = loss_and_grads(Ft, W, pairs, DIMS, apply_m=A)
    rng = np.random.default_rng(44)
    h = 1e-6
    for _ in range(6):
        l = rng.integers(len(W))
        idx = tuple(rng.integers(s) for s in W[l].shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][idx] += h * unit
            Wm[l][idx] -= h * unit
            fd = (loss_and_grads(Ft, Wp, pairs, DIMS, A)[0] - loss_and_grads(Ft, Wm, pairs, DIMS, A)[0]) / (2 * h)
            an = 2 * (grads[l][idx].real if part == "re" else grads[l][idx].imag)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def _system(dims, seed, m=0.1):
    fat, lng = fat_field(dims, seed), random_su3_field(dims, seed + 1)
    return fat, lng, (lambda v: apply_m(fat, lng, v, dims, m))


def test_fcg_identity_preconditioner_is_cg():
    dims = (4, 4, 4, 4)
    _, _, A = _system(dims, 20)
    b = gaussian_source(dims, 21)[0]
    ref = cg(A, b, tol=1e-10, record=15)
    res = fcg(A, lambda r: r.copy(), b, tol=1e-10, record=15)
    assert res.converged and not res.fell_back
    np.testing.assert_allclose(np.real(res.alphas), ref.alphas, rtol=1e-8)
    assert abs(res.iters - ref.iters) <= 1


def test_fcg_exact_inverse_converges_in_one_step():
    dims = (2, 2, 2, 2)
    fat, lng, A = _system(dims, 22)
    M = dense.dense_normal_operator(fat, lng, dims, 0.1)
    Minv = np.linalg.inv(M)
    b = gaussian_source(dims, 23)[0]
    res = fcg(A, lambda r: (Minv @ r.reshape(-1)).reshape(r.shape), b, tol=1e-10)
    assert res.fcg_iters == 1 and res.converged


def test_fcg_falls_back_when_preconditioner_stalls():
    """A preconditioner that returns noise stalls; plain CG then finishes to the same true residual."""
    dims = (4, 4, 4, 4)
    _, _, A = _system(dims, 24, m=0.05)
    b = gaussian_source(dims, 25)[0]
    rng = np.random.default_rng(26)
    noise = lambda r: 1e-8 * (rng.standard_normal(r.shape) + 1j * rng.standard_normal(r.shape))
    res = fcg(A, noise, b, tol=1e-10, stall_window=5)
    assert res.fell_back and res.converged and res.true_resid <= 1e-10


def test_tied_network_is_hermitian_positive():
    """N = K^dag K built from the adjoint layers is Hermitian and positive semi-definite."""
    fat = fat_field(DIMS, 50)
    Ft = folded_fat(fat, DIMS)
    W = hermitian_weights(init_weights([1, 3, 3], 51, scale=1.0))
    u = gaussian_source(DIMS, 52)[0]
    v = gaussian_source(DIMS, 53)[0]
    a = np.vdot(u, net_forward(Ft, W, v, DIMS))
    b = np.conj(np.vdot(v, net_forward(Ft, W, u, DIMS)))
    assert abs(a - b) <= 1e-12 * abs(a)
    q = np.vdot(v, net_forward(Ft, W, v, DIMS))
    assert q.real > 0 and abs(q.imag) <= 1e-12 * q.real
