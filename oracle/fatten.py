"""Link fattening: the one-hop (fat) and three-hop (long) link fields of the improved action, built from a
thin gauge field.  TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs on a MILC ensemble whose improved staggered action (Sec. 1 and Sec. 2: the fine 28^3x96
lattice, the MILC/CPS setting) carries fat one-hop links and three-hop Naik links, but it does not state
how the fat links are made.  The recipe taken here is the published asqtad construction (K. Orginos,
D. Toussaint and R. L. Sugar, Phys. Rev. D 60, 054503 (1999); G. P. Lepage, Phys. Rev. D 59, 074502
(1999)), written out as a sum over explicit lattice paths from n to n + mu:

  V_mu(n) = c_1 U_mu(n)                                              (1 path)
          + c_3 sum_{+-nu}           [nu, mu, -nu]                    (6 three-link staples)
          + c_5 sum_{+-nu, +-rho}     [nu, rho, mu, -rho, -nu]         (24 five-link staples, nu != rho)
          + c_7 sum_{+-nu,+-rho,+-si} [nu, rho, si, mu, -si, -rho, -nu] (48 seven-link staples, all distinct)
          + c_L sum_{+-nu}           [nu, nu, mu, -nu, -nu]           (6 Lepage paths)

  W_mu(n) = U_mu(n) U_mu(n + mu) U_mu(n + 2 mu)                      (the three-hop product)

Every transverse direction is different from mu.  A path is the ordered product of its links: a step
+nu from site m multiplies by U_nu(m), a step -nu from m by U_nu(m - nu)^dagger.  Coefficients
(for links without the staggered phases, which the Dirac operator adds later):

  c_1 = 5/8, c_3 = 1/16, c_5 = 1/64, c_7 = 1/384, c_L = -1/16,

each path of length l scaled by u0^(1 - l) for the tadpole factor u0 (u0 = 1: no tadpole improvement).
The three-hop links W enter the operator with c_N = -1/(24 u0^2); that coefficient is applied where the
links are packed, not here.  With unit links the fat link is (5/8 + 6/16 + 24/64 + 48/384 - 6/16) = 9/8
times the identity, the tree-level normalisation of the Naik-improved derivative.

The gauge field is periodic in every direction (the fermion's antiperiodic time is a sign of the
operator, folded in at packing).  Layout as everywhere: [4][Lt][Lz][Ly][Lx][3][3].
"""
from __future__ import annotations

from itertools import permutations

import numpy as np

# (name, coefficient at u0 = 1, path length)
ASQTAD = {"one": (5.0 / 8.0, 1), "three": (1.0 / 16.0, 3), "five": (1.0 / 64.0, 5),
          "seven": (1.0 / 384.0, 7), "lepage": (-1.0 / 16.0, 5)}


def asqtad_coeffs(u0: float = 1.0) -> dict:
    """Path-class coefficients c * u0^(1 - length)."""
    return {k: c * u0 ** (1 - l) for k, (c, l) in ASQTAD.items()}


def paths(mu: int):
    """The fat-link paths of direction mu as (class, [(direction, +1 or -1), ...])."""
    others = [nu for nu in range(4) if nu != mu]
    out = [("one", [(mu, 1)])]
    for nu in others:
        for s in (1, -1):
            out.append(("three", [(nu, s), (mu, 1), (nu, -s)]))
    for nu, rho in permutations(others, 2):
        for s1 in (1, -1):
            for s2 in (1, -1):
                out.append(("five", [(nu, s1), (rho, s2), (mu, 1), (rho, -s2), (nu, -s1)]))
    for nu, rho, si in permutations(others, 3):
        for s1 in (1, -1):
            for s2 in (1, -1):
                for s3 in (1, -1):
                    out.append(("seven", [(nu, s1), (rho, s2), (si, s3), (mu, 1), (si, -s3), (rho, -s2),
                                          (nu, -s1)]))
    for nu in others:
        for s in (1, -1):
            out.append(("lepage", [(nu, s), (nu, s), (mu, 1), (nu, -s), (nu, -s)]))
    return out


def _shifted(field: np.ndarray, off) -> np.ndarray:
    """f(n + off) for a [Lt][Lz][Ly][Lx]... field (periodic)."""
    return np.roll(field, shift=(-off[3], -off[2], -off[1], -off[0]), axis=(0, 1, 2, 3))


def path_product(U: np.ndarray, steps) -> tuple:
    """Field P(n) = ordered product of the links along `steps` from n, and the path's end offset."""
    off = [0, 0, 0, 0]
    P = None
    for nu, s in steps:
        if s > 0:
            link = _shifted(U[nu], off)
            off[nu] += 1
        else:
            off[nu] -= 1
            link = np.conj(np.swapaxes(_shifted(U[nu], off), -1, -2))
        P = link.copy() if P is None else np.einsum("...ab,...bc->...ac", P, link)
    return P, off


def fat_links(U: np.ndarray, dims, u0: float = 1.0) -> np.ndarray:
    """V_mu(n) for every mu and site: the coefficient-weighted sum of the 85 path products."""
    c = asqtad_coeffs(u0)
    V = np.zeros_like(U)
    for mu in range(4):
        for cls, steps in paths(mu):
            P, off = path_product(U, steps)
            assert off == [1 if d == mu else 0 for d in range(4)], (cls, steps, off)
            V[mu] += c[cls] * P
    return V


def long_links(U: np.ndarray, dims) -> np.ndarray:
    """W_mu(n) = U_mu(n) U_mu(n + mu) U_mu(n + 2 mu)."""
    W = np.empty_like(U)
    for mu in range(4):
        W[mu], off = path_product(U, [(mu, 1)] * 3)
        assert off[mu] == 3
    return W


def fat_link_at(U: np.ndarray, dims, site, mu: int, u0: float = 1.0) -> np.ndarray:
    """V_mu at one site (x, y, z, t), walking every path with scalar index arithmetic (for lattices too big
    for fat_links; the same definition, one site at a time)."""
    c = asqtad_coeffs(u0)
    out = np.zeros((3, 3), dtype=np.complex128)
    for cls, steps in paths(mu):
        out += c[cls] * _walk(U, dims, site, steps)
    return out


def long_link_at(U: np.ndarray, dims, site, mu: int) -> np.ndarray:
    return _walk(U, dims, site, [(mu, 1)] * 3)


def _walk(U, dims, site, steps) -> np.ndarray:
    m = list(site)
    P = np.eye(3, dtype=np.complex128)
    for nu, s in steps:
        if s > 0:
            P = P @ U[nu, m[3], m[2], m[1], m[0]]
            m[nu] = (m[nu] + 1) % dims[nu]
        else:
            m[nu] = (m[nu] - 1) % dims[nu]
            P = P @ U[nu, m[3], m[2], m[1], m[0]].conj().T
    return P


__all__ = ["ASQTAD", "asqtad_coeffs", "paths", "path_product", "fat_links", "long_links", "fat_link_at",
           "long_link_at"]
