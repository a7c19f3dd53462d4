"""Conjugate gradient, paper Fig. 1, in complex128.

The loop is the figure's, step for step:
    r = b - A x ; d = r ; delta_new = r^dag r
    while i < N_dim and delta_new > eps^2 * delta_0:
        alpha = delta_new / d^dag A d
        x = x + alpha d
        r = r - alpha A d
        delta_old = delta_new ; delta_new = r^dag r
        beta = delta_new / delta_old
        d = r + beta d

Readings where the paper is silent:
  * The stopping test uses eps^2 * ||b||^2 in place of eps^2 * delta_0, which is
    the same thing for x0 = 0, and eps bounds the norm (not its square).
  * d^dag A d is real for Hermitian A; its real part is used.
  * After the loop the true residual ||b - A x|| / ||b|| is computed; if it
    exceeds eps the loop restarts from the current x (at most max_restarts times).
  * N_dim defaults to the dimension 3V/2 of the even-site space.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    true_resid: float
    converged: bool
    restarts: int = 0
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    resid_history: list = field(default_factory=list)


def cg(apply_a, b: np.ndarray, tol: float = 1e-10, x0=None, max_iter: int | None = None,
       max_restarts: int = 5, record: int = 0) -> CGResult:
    """Solve A x = b for Hermitian positive-definite A given as a callable.

    record > 0 keeps the first `record` alphas and betas (for iterate-level checks).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    n_dim = b.size if max_iter is None else max_iter
    b2 = float(np.vdot(b, b).real)
    res = CGResult(x=x, iters=0, true_resid=np.inf, converged=False)
    if b2 == 0.0:
        res.x = np.zeros_like(b)
        res.true_resid = 0.0
        res.converged = True
        return res
    for attempt in range(max_restarts + 1):
        r = b - apply_a(x)
        d = r.copy()
        delta_new = float(np.vdot(r, r).real)
        i = 0
        while i < n_dim and delta_new > tol * tol * b2:
            Ad = apply_a(d)
            dAd = np.vdot(d, Ad)
            alpha = delta_new / dAd.real
            x = x + alpha * d
            r = r - alpha * Ad
            delta_old = delta_new
            delta_new = float(np.vdot(r, r).real)
            beta = delta_new / delta_old
            d = r + beta * d
            i += 1
            if len(res.alphas) < record:
                res.alphas.append(alpha)
                res.betas.append(beta)
            res.resid_history.append(np.sqrt(delta_new / b2))
        res.iters += i
        rt = b - apply_a(x)
        res.true_resid = float(np.sqrt(np.vdot(rt, rt).real / b2))
        res.restarts = attempt
        if res.true_resid <= tol:
            res.converged = True
            break
    res.x = x
    return res


def true_residual(apply_a, b: np.ndarray, x: np.ndarray) -> float:
    """||b - A x|| / ||b||."""
    r = b - apply_a(x)
    return float(np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real))


def true_residuals(apply_a, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """||b_r - A x_r|| / ||b_r|| for every right-hand side r of b, x: [nrhs][...] (A applied to all at once)."""
    r = b - apply_a(x)
    axes = tuple(range(1, b.ndim))
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=axes) / np.sum(np.abs(b) ** 2, axis=axes))
