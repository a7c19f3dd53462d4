"""The staggered Dirac operator, its even-odd blocks and the normal operator.

Definition (paper Sec. 2, Eqs. (4)-(5), with the staggered phases folded into the
links as the paper states, and the three-hop Naik term of the improved action
added with coefficient c_N):

  (D chi)(n) = sum_mu eta_mu(n) * [ s(n,1) F_mu(n) chi(n+mu)
                                   - s(n-mu,1) F_mu(n-mu)^dag chi(n-mu)
                                   + c_N ( s(n,3) W_mu(n) chi(n+3mu)
                                           - s(n-3mu,3) W_mu(n-3mu)^dag chi(n-3mu) ) ]

F are the one-hop (fat) links, W the three-hop (long) links, s(m,k) the boundary
sign of the forward hop of length k that starts at m (geometry.hop_sign).  With
W = 0 this is the paper's Eq. (5).  Contributions that land on the same site
(extent <= 6) add.

Normal operator (paper Eq. (3) written on even sites; the paper writes
A = -D^2 + m^2, the form used here is 4 m^2 - D_eo D_oe, i.e. the paper's m is
twice this m):

  M chi_e = 4 m^2 chi_e - D_eo (D_oe chi_e).
"""
from __future__ import annotations

import numpy as np

from .geometry import embed, eta, hop_sign, restrict, shift, coords

NAIK_COEFF = -1.0 / 24.0


def _matvec(U: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Per-site 3x3 matrix times colour vector."""
    return np.einsum("...ab,...b->...a", U, v)


def _dagger_matvec(U: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Per-site U^dagger times colour vector."""
    return np.einsum("...ba,...b->...a", U.conj(), v)


def dslash_full(fat: np.ndarray, lng, chi: np.ndarray, dims, antiperiodic_t: bool = True,
                naik: float = NAIK_COEFF) -> np.ndarray:
    """D chi on the full lattice.  fat, lng: [4][Lt][Lz][Ly][Lx][3][3]; chi: [Lt][Lz][Ly][Lx][3].

    lng=None (or naik=0) drops the three-hop term, leaving the paper's one-hop Eq. (5).
    """
    out = np.zeros_like(chi, dtype=np.complex128)
    terms = [(1, fat, 1.0)]
    if lng is not None and naik != 0.0:
        terms.append((3, lng, naik))
    for mu in range(4):
        eta_mu = eta(mu, dims)[..., None]
        for k, U, c in terms:
            s = hop_sign(mu, k, dims, antiperiodic_t)[..., None]
            forward = s * _matvec(U[mu], shift(chi, mu, k))
            # backward(n) = s(n-k mu, k) U(n-k mu)^dag chi(n-k mu): build at the start
            # site m, then move it forward by k so that it sits at n = m + k mu.
            backward = shift(s * _dagger_matvec(U[mu], chi), mu, -k)
            out += c * eta_mu * (forward - backward)
    return out


def dslash_eo(fat, lng, chi_half: np.ndarray, dims, out_parity: int, antiperiodic_t: bool = True,
              naik: float = NAIK_COEFF) -> np.ndarray:
    """D_{p,1-p}: input [V/2][3] on parity 1-p, output [V/2][3] on parity p."""
    full = embed(chi_half, dims, 1 - out_parity)
    return restrict(dslash_full(fat, lng, full, dims, antiperiodic_t, naik), dims, out_parity)


def apply_m(fat, lng, chi_e: np.ndarray, dims, mass: float, antiperiodic_t: bool = True,
            naik: float = NAIK_COEFF) -> np.ndarray:
    """M chi_e = 4 m^2 chi_e - D_eo D_oe chi_e (even sites)."""
    t_o = dslash_eo(fat, lng, chi_e, dims, 1, antiperiodic_t, naik)
    return 4.0 * mass * mass * chi_e - dslash_eo(fat, lng, t_o, dims, 0, antiperiodic_t, naik)


def dslash_at_sites(fat, lng, chi_half: np.ndarray, dims, out_parity: int, cbs,
                    antiperiodic_t: bool = True, naik: float = NAIK_COEFF) -> np.ndarray:
    """(D_{p,1-p} chi)(n) evaluated one output site at a time, for the sites cbs of parity p.

    Reads only the links and input components each site needs, so it works on
    lattices too big for dslash_full.  chi_half is [V/2][3] or [nrhs][V/2][3];
    returns [len(cbs)][3] or [nrhs][len(cbs)][3].
    """
    Lx, Ly, Lz, Lt = dims
    L = np.array(dims)
    cbs = np.asarray(cbs, dtype=np.int64)
    xh = cbs % (Lx // 2)
    rest = cbs // (Lx // 2)
    y = rest % Ly
    rest //= Ly
    z = rest % Lz
    t = rest // Lz
    x = 2 * xh + ((y + z + t + out_parity) % 2)
    n = np.stack([x, y, z, t], axis=1)               # [S][4]
    multi = chi_half.ndim == 3

    def chi_at(m):                                   # m: [S][4], parity 1-p -> [S][3] or [nrhs][S][3]
        lex = m[:, 0] + Lx * (m[:, 1] + Ly * (m[:, 2] + Lz * m[:, 3]))
        return chi_half[:, lex // 2] if multi else chi_half[lex // 2]

    def link(U, mu, m):
        return U[mu, m[:, 3], m[:, 2], m[:, 1], m[:, 0]]

    def sign(mu, k, m):
        if mu != 3 or not antiperiodic_t:
            return np.ones(len(m))
        return np.where(((m[:, 3] + k) // Lt) % 2 == 0, 1.0, -1.0)

    out = np.zeros(chi_half.shape[:-2] + (len(cbs), 3), dtype=np.complex128)
    terms = [(1, fat, 1.0)]
    if lng is not None and naik != 0.0:
        terms.append((3, lng, naik))
    for mu in range(4):
        e = np.where(n[:, :mu].sum(axis=1) % 2 == 0, 1.0, -1.0)
        for k, U, c in terms:
            fwd = n.copy()
            fwd[:, mu] = (n[:, mu] + k) % L[mu]
            bwd = n.copy()
            bwd[:, mu] = (n[:, mu] - k) % L[mu]
            term = sign(mu, k, n)[:, None] * _matvec(link(U, mu, n), chi_at(fwd))
            term -= sign(mu, k, bwd)[:, None] * _dagger_matvec(link(U, mu, bwd), chi_at(bwd))
            out += c * e[:, None] * term
    return out


def dslash_eo_chunked(fat, lng, chi_half: np.ndarray, dims, out_parity: int, chunk: int = 1 << 16,
                      workers: int = 1, antiperiodic_t: bool = True, naik: float = NAIK_COEFF) -> np.ndarray:
    """D_{p,1-p} on every output site, computed by dslash_at_sites over consecutive chunks of sites.

    The same definition as dslash_eo with memory bounded by the chunk; chunks are independent, so
    `workers` threads may evaluate them concurrently (NumPy's gathers and products release the GIL).
    chi_half is [V/2][3] or [nrhs][V/2][3].
    """
    from concurrent.futures import ThreadPoolExecutor

    half = chi_half.shape[-2]
    out = np.empty(chi_half.shape, dtype=np.complex128)

    def run(c0):
        cbs = np.arange(c0, min(half, c0 + chunk))
        out[..., c0:c0 + len(cbs), :] = dslash_at_sites(fat, lng, chi_half, dims, out_parity, cbs,
                                                        antiperiodic_t, naik)

    starts = range(0, half, chunk)
    if workers <= 1:
        for c0 in starts:
            run(c0)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(run, starts))
    return out


def apply_m_chunked(fat, lng, chi_e: np.ndarray, dims, mass, chunk: int = 1 << 16, workers: int = 1,
                    antiperiodic_t: bool = True, naik: float = NAIK_COEFF) -> np.ndarray:
    """M chi_e = 4 m^2 chi_e - D_eo D_oe chi_e with the chunked operator; chi_e [V/2][3] or [nrhs][V/2][3],
    mass a scalar or one per right-hand side."""
    t_o = dslash_eo_chunked(fat, lng, chi_e, dims, 1, chunk, workers, antiperiodic_t, naik)
    m = np.asarray(mass, dtype=np.float64)
    m4 = (4.0 * m * m).reshape(m.shape + (1, 1)) if m.ndim else 4.0 * m * m
    return m4 * chi_e - dslash_eo_chunked(fat, lng, t_o, dims, 0, chunk, workers, antiperiodic_t, naik)


def gauge_transform_links(fat, lng, g, dims):
    """U_mu(n) -> g(n) U_mu(n) g(n+k mu)^dag for the one-hop (k=1) and three-hop (k=3) fields."""
    def tr(U, k):
        out = np.empty_like(U)
        for mu in range(4):
            g_fwd = shift(g, mu, k)
            out[mu] = np.einsum("...ab,...bc,...dc->...ad", g, U[mu], g_fwd.conj())
        return out
    return tr(fat, 1), (None if lng is None else tr(lng, 3))


def pure_gauge_links(g, dims):
    """F_mu(n) = g(n) g(n+mu)^dag and W_mu(n) = g(n) g(n+3mu)^dag."""
    Lx, Ly, Lz, Lt = dims
    fat = np.empty((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    lng = np.empty_like(fat)
    for mu in range(4):
        fat[mu] = np.einsum("...ab,...cb->...ac", g, shift(g, mu, 1).conj())
        lng[mu] = np.einsum("...ab,...cb->...ac", g, shift(g, mu, 3).conj())
    return fat, lng


def colour_rotate(g, chi):
    """(g chi)(n) = g(n) chi(n) for a full field."""
    return _matvec(g, chi)


__all__ = ["dslash_full", "dslash_eo", "apply_m", "dslash_at_sites", "dslash_eo_chunked", "apply_m_chunked",
           "gauge_transform_links",
           "pure_gauge_links", "colour_rotate", "coords", "NAIK_COEFF"]
