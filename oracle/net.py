"""Gauge-covariant linear network, the learned preconditioner of the flexible CG (complex128).

The paper has no preconditioner; this is the project's third change to its
method.  A layer maps C_in colour-vector channels on the full lattice to C_out:

    y_c(n) = sum_{c'} [ W_0[c][c'] psi_c'(n) + sum_{d=1..8} W_d[c][c'] (T_d psi_c')(n) ]

with the parallel transports along the one-hop (fat) links, phases and boundary
signs folded in as in the Dirac operator (F~_mu(n) = eta_mu(n) s(n,1) F_mu(n)):

    d = 1..4 (+mu, mu = d-1):  (T_d psi)(n) = F~_mu(n) psi(n + mu)
    d = 5..8 (-mu, mu = d-5):  (T_d psi)(n) = F~_mu(n - mu)^dag psi(n - mu)

The network embeds an even-site vector on the full lattice (zero on odd sites),
applies its layers (channels 1 -> C -> ... -> C -> 1) and restricts the result to
the even sites.  It is linear in its input and gauge covariant: with
F_mu(n) -> g(n) F_mu(n) g(n+mu)^dag it satisfies N[U^g](g r) = g N[U](r).

Gradients: for the real loss L, G = dL/d conj(.) is propagated backwards; a layer's
input gradient is L^dag G (T_{+mu}^dag = T_{-mu}), and the weight gradient is
dL/d conj(W_d[c][c']) = sum_{n,a} G_c(n)_a conj((T_d psi_c')(n)_a).  For a real
optimiser the gradient with respect to (Re W, Im W) is 2 (Re G_W, Im G_W).
"""
from __future__ import annotations

import numpy as np

from .geometry import embed, eta, hop_sign, restrict

NDIR = 9  # identity + 8 transports


def folded_fat(fat, dims, antiperiodic_t: bool = True) -> np.ndarray:
    """F~_mu(n) = eta_mu(n) s(n,1) F_mu(n)."""
    out = np.empty_like(fat)
    for mu in range(4):
        c = eta(mu, dims) * hop_sign(mu, 1, dims, antiperiodic_t)
        out[mu] = c[..., None, None] * fat[mu]
    return out


def transport(Ft, psi, d: int):
    """(T_d psi) for d = 1..8 on a full field [..., Lt, Lz, Ly, Lx, 3] (leading channel axes allowed)."""
    if d <= 4:
        mu = d - 1
        # the lattice axis of direction mu, counted from the colour axis at the end
        return np.einsum("...ab,...b->...a", Ft[mu], np.roll(psi, -1, axis=psi.ndim - 2 - mu))
    mu = d - 5
    v = np.einsum("...ba,...b->...a", Ft[mu].conj(), psi)
    return np.roll(v, 1, axis=psi.ndim - 2 - mu)


def transport_adjoint(Ft, phi, d: int):
    """T_d^dag phi: the adjoint of a forward transport is the backward one and vice versa."""
    return transport(Ft, phi, d + 4 if d <= 4 else d - 4)


def layer_forward(Ft, psi, W):
    """psi: [C_in][Lt][Lz][Ly][Lx][3]; W: [9][C_out][C_in] -> y [C_out][...][3]."""
    y = np.einsum("oi,i...->o...", W[0], psi)
    for d in range(1, NDIR):
        y += np.einsum("oi,i...->o...", W[d], transport(Ft, psi, d))
    return y


def layer_backward(Ft, psi, W, g_y):
    """Given G_y = dL/d conj(y), return (G_psi, G_W) with G_W [9][C_out][C_in]."""
    gW = np.empty_like(W)
    g_psi = np.zeros_like(psi)
    for d in range(NDIR):
        t = psi if d == 0 else transport(Ft, psi, d)
        gW[d] = g_y.reshape(len(g_y), -1) @ t.reshape(len(t), -1).conj().T
        back = np.einsum("oi,o...->i...", W[d].conj(), g_y)
        g_psi += back if d == 0 else transport_adjoint(Ft, back, d)
    return g_psi, gW


def net_forward(Ft, weights, r_e, dims, keep=False):
    """N(r): embed the even-site vector, apply the layers, restrict to even sites."""
    psi = embed(r_e, dims, 0)[None]
    acts = [psi]
    for W in weights:
        psi = layer_forward(Ft, psi, W)
        acts.append(psi)
    out = restrict(psi[0], dims, 0)
    return (out, acts) if keep else out


def net_backward(Ft, weights, acts, g_out_e, dims):
    """Weight gradients G_W per layer for the output gradient g_out_e = dL/d conj(N(r)) on even sites."""
    g = embed(g_out_e, dims, 0)[None]
    grads = [None] * len(weights)
    for l in range(len(weights) - 1, -1, -1):
        g, grads[l] = layer_backward(Ft, acts[l], weights[l], g)
    return grads


def loss_and_grads(Ft, weights, pairs, dims, apply_m=None):
    """Training loss and dL/d conj(W) per layer.

    apply_m None (solution loss): L = sum_i ||N(b_i) - x_i||^2 / ||x_i||^2, output gradient (N(b) - x)/||x||^2.
    apply_m given (residual loss): L = sum_i ||M N(b_i) - b_i||^2 / ||b_i||^2 (equal to
    ||M (N(b_i) - x_i)||^2 / ||b_i||^2 for exact pairs); M is Hermitian, so the output gradient is
    M (M N(b) - b) / ||b||^2.
    """
    total = 0.0
    grads = [np.zeros_like(W) for W in weights]
    for b, x in pairs:
        out, acts = net_forward(Ft, weights, b, dims, keep=True)
        if apply_m is None:
            nx = float(np.vdot(x, x).real)
            res = out - x
            total += float(np.vdot(res, res).real) / nx
            g = res / nx
        else:
            nb = float(np.vdot(b, b).real)
            res = apply_m(out) - b
            total += float(np.vdot(res, res).real) / nb
            g = apply_m(res) / nb
        for acc, gl in zip(grads, net_backward(Ft, weights, acts, g, dims)):
            acc += gl
    return total, grads


def init_weights(channels, seed: int, scale: float = 0.1):
    """Random complex weights for the channel sequence, e.g. [1, 8, 8, 8, 1]."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = scale / np.sqrt(NDIR * cin)
        out.append(s * (rng.standard_normal((NDIR, cout, cin)) + 1j * rng.standard_normal((NDIR, cout, cin))))
    return out


def adjoint_layer_weights(W):
    """Weights of the adjoint layer: adj(W)[d'][a][b] = conj(W[d][b][a]), d' the opposite direction."""
    opp = [0, 5, 6, 7, 8, 1, 2, 3, 4]
    A = np.empty((9, W.shape[2], W.shape[1]), dtype=W.dtype)
    for d in range(9):
        A[opp[d]] = W[d].conj().T
    return A


def hermitian_weights(K):
    """Layers of N = K^dag K: the layers of K followed by their adjoints in reverse order."""
    return list(K) + [adjoint_layer_weights(W) for W in reversed(K)]
