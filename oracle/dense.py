"""Dense matrix of the staggered operator, built entry by entry with scalar loops.

Written independently of the vectorised operator in dslash.py (no NumPy rolls,
no shared helpers beyond the conventions of geometry.py restated inline) so
that each can check the other.  For lattices of at most a few hundred sites.

Row/column index of (site n, colour a) is 3 * lex(n) + a with
lex = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import itertools

import numpy as np

NAIK_COEFF = -1.0 / 24.0


def dense_dslash(fat, lng, dims, antiperiodic_t: bool = True, naik: float = NAIK_COEFF) -> np.ndarray:
    """3V x 3V matrix of D (Eq. (5) with folded phases and the three-hop term)."""
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)
    V = Lx * Ly * Lz * Lt
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)

    def lex(c):
        return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))

    def link(U, mu, c):
        return U[mu][c[3]][c[2]][c[1]][c[0]]

    hops = [(1, fat, 1.0)]
    if lng is not None and naik != 0.0:
        hops.append((3, lng, naik))
    for n in itertools.product(range(Lx), range(Ly), range(Lz), range(Lt)):
        row = 3 * lex(n)
        for mu in range(4):
            eta = -1.0 if sum(n[:mu]) % 2 else 1.0
            for k, U, c in hops:
                # forward hop n -> n + k mu; the sign counts wraps of the time direction
                f = list(n)
                wraps = (n[mu] + k) // L[mu]
                f[mu] = (n[mu] + k) % L[mu]
                s_f = (-1.0) ** wraps if (mu == 3 and antiperiodic_t) else 1.0
                col = 3 * lex(f)
                D[row:row + 3, col:col + 3] += c * eta * s_f * link(U, mu, n)
                # backward hop: the link that starts at m = n - k mu and ends at n
                m = list(n)
                m[mu] = (n[mu] - k) % L[mu]
                wraps_m = (m[mu] + k) // L[mu]
                s_b = (-1.0) ** wraps_m if (mu == 3 and antiperiodic_t) else 1.0
                col = 3 * lex(m)
                D[row:row + 3, col:col + 3] -= c * eta * s_b * link(U, mu, m).conj().T
    return D


def parity_indices(dims, par: int) -> np.ndarray:
    """Dense row indices (3 lex + a) of the sites of parity par, in lexicographic order."""
    Lx, Ly, Lz, Lt = dims
    idx = []
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    if (x + y + z + t) % 2 == par:
                        l3 = 3 * (x + Lx * (y + Ly * (z + Lz * t)))
                        idx.extend([l3, l3 + 1, l3 + 2])
    return np.array(idx)


def dense_normal_operator(fat, lng, dims, mass: float, antiperiodic_t: bool = True,
                          naik: float = NAIK_COEFF) -> np.ndarray:
    """Dense M = 4 m^2 - D_eo D_oe on the even sites ((3V/2) x (3V/2))."""
    D = dense_dslash(fat, lng, dims, antiperiodic_t, naik)
    e = parity_indices(dims, 0)
    o = parity_indices(dims, 1)
    D_eo = D[np.ix_(e, o)]
    D_oe = D[np.ix_(o, e)]
    return 4.0 * mass * mass * np.eye(len(e)) - D_eo @ D_oe
