"""Point-source propagators and the staggered pion correlator, built on the even-site solve.

Test infrastructure: only tests/, the smoke check and the bench's CPU-baseline leg use this module.

The paper's CG is run in production to compute hadron spectra (its closing remarks); the step after the
solve is the quark propagator from point sources on one gauge field.  With the full staggered operator
M = 2m + D (D anti-Hermitian, so that M^dag M = 4m^2 - D^2 is the normal operator of Eq. (3) in the form
4m^2 - D_eo D_oe on even sites; the paper's m is twice this m), a source delta on an even site gives

    G = M^{-1} delta = M^dag (M M^dag)^{-1} delta = (2m - D) chi,   chi_e = (4m^2 - D_eo D_oe)^{-1} delta_e,

that is  G_e = 2m chi_e  and  G_o = -D_oe chi_e  (chi vanishes on odd sites).  The Goldstone-pion
correlator sums |G|^2 over a time slice, over the sink colour and over the three source colours:

    C(t) = sum_{x with time t} sum_{a, c} |G^(c)(x)_a|^2.

Because M M^dag is the normal operator, sum_t C(t) = sum_c (A_e^{-1})_{cc}(x0, x0) = sum_c chi^(c)(x0)_c,
an identity the tests use as a pin that does not run through this module.
"""
from __future__ import annotations

import numpy as np

from stag_inputs import point_sources  # noqa: F401  (the unit sources are inputs, shared with the GPU side)

from .cg import cg
from .dslash import NAIK_COEFF, apply_m, dslash_eo
from .geometry import embed, parity


def even_solutions(fat, lng, dims, mass: float, sources, tol: float = 1e-12, naik: float = NAIK_COEFF):
    """chi_e for every source row (plain CG of Fig. 1 on the normal operator)."""
    return np.stack([cg(lambda v: apply_m(fat, lng, v, dims, mass, naik=naik), b, tol=tol).x for b in sources])


def propagator(fat, lng, dims, mass: float, chi_e: np.ndarray, naik: float = NAIK_COEFF):
    """(G_e, G_o) = (2m chi_e, -D_oe chi_e) for solutions chi_e [n][V/2][3]."""
    g_e = 2.0 * mass * chi_e
    g_o = np.stack([-dslash_eo(fat, lng, c, dims, 1, naik=naik) for c in chi_e])
    return g_e, g_o


def full_field(g_e: np.ndarray, g_o: np.ndarray, dims) -> np.ndarray:
    """Even and odd halves -> full field [Lt][Lz][Ly][Lx][3]."""
    return embed(g_e, dims, 0) + embed(g_o, dims, 1)


def correlator(g_e: np.ndarray, g_o: np.ndarray, dims) -> np.ndarray:
    """C[s][t] for propagators given as 3 consecutive rows (source colours) per source."""
    Lt = dims[3]
    n = g_e.shape[0] // 3
    par = parity(dims)
    t_of = np.broadcast_to(np.arange(Lt)[:, None, None, None], par.shape)
    t_e = t_of[par == 0]
    t_o = t_of[par == 1]
    C = np.zeros((n, Lt))
    for s in range(n):
        for c in range(3):
            w_e = np.sum(np.abs(g_e[3 * s + c]) ** 2, axis=1)
            w_o = np.sum(np.abs(g_o[3 * s + c]) ** 2, axis=1)
            C[s] += np.bincount(t_e, weights=w_e, minlength=Lt) + np.bincount(t_o, weights=w_o, minlength=Lt)
    return C
