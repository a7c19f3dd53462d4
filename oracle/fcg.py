"""Flexible CG with a (possibly nonlinear, non-Hermitian) preconditioner and a stall fallback.

The project's third change to the paper's Fig. 1 loop: each iteration applies a
preconditioner z = N(r) and makes the new direction A-orthogonal to the previous
one (flexible CG with one stored direction, after Notay):

    beta_k = -<A d_{k-1}, z_k> / <d_{k-1}, A d_{k-1}>,   d_k = z_k + beta_k d_{k-1},

with the exact line-search step alpha_k = <d_k, r_k> / <d_k, A d_k> (complex in
general; <d, A d> is real for Hermitian A).  With N = identity this is the CG of
Fig. 1 iterate for iterate (in exact arithmetic, and to the iteration in double
precision); with N = A^{-1} it converges in one step.  The Polak-Ribiere form
beta_k = <z_k, r_k - r_{k-1}> / <z_{k-1}, r_{k-1}> is equal in exact arithmetic but
lost 40% in iterations to CG with N = identity in double precision, so the
explicit orthogonalisation is used.

Fallback: every w iterations (the stall window) the smallest ||r|| seen so far is
compared with the smallest one seen w iterations earlier; if it did not fall below
stall_ratio times that value, the preconditioner is abandoned and plain CG
(oracle.cg) finishes from the current x.  (The residual of a preconditioned CG need
not fall monotonically, so the running minimum is compared, not ||r_k||.)
The result is judged, like every solve, by its true residual.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .cg import cg


@dataclass
class FCGResult:
    x: np.ndarray
    iters: int
    true_resid: float
    converged: bool
    fell_back: bool = False
    fcg_iters: int = 0
    alphas: list = field(default_factory=list)
    resid_history: list = field(default_factory=list)


def fcg(apply_a, precond, b, tol=1e-10, x0=None, max_iter=None, stall_window=10, stall_ratio=0.9,
        record=0) -> FCGResult:
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    n_dim = b.size if max_iter is None else max_iter
    b2 = float(np.vdot(b, b).real)
    res = FCGResult(x=x, iters=0, true_resid=np.inf, converged=False)
    r = b - apply_a(x)
    norms = [np.sqrt(float(np.vdot(r, r).real))]
    d = precond(r)
    k = 0
    while k < n_dim and norms[-1] ** 2 > tol * tol * b2:
        Ad = apply_a(d)
        alpha = np.vdot(d, r) / np.vdot(d, Ad).real
        x = x + alpha * d
        r = r - alpha * Ad
        k += 1
        if len(res.alphas) < record:
            res.alphas.append(alpha)
        norms.append(np.sqrt(float(np.vdot(r, r).real)))
        res.resid_history.append(norms[-1] / np.sqrt(b2))
        if norms[-1] ** 2 <= tol * tol * b2:
            break
        if k % stall_window == 0 and min(norms) > stall_ratio * min(norms[:len(norms) - stall_window]):
            res.fell_back = True
            break
        z = precond(r)
        beta = -np.vdot(Ad, z) / np.vdot(d, Ad).real
        d = z + beta * d
    res.fcg_iters = k
    res.iters = k
    if res.fell_back:
        rest = cg(apply_a, b, tol=tol, x0=x)
        res.x, res.iters = rest.x, k + rest.iters
        res.true_resid, res.converged = rest.true_resid, rest.converged
        return res
    rt = b - apply_a(x)
    res.x = x
    res.true_resid = float(np.sqrt(np.vdot(rt, rt).real / b2))
    res.converged = res.true_resid <= tol
    if not res.converged and k < n_dim:
        rest = cg(apply_a, b, tol=tol, x0=x)
        res.x, res.iters = rest.x, k + rest.iters
        res.true_resid, res.converged = rest.true_resid, rest.converged
    return res
