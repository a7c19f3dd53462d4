"""Reference for the low-precision Dslash: the operator evaluated exactly (FP64) on rounded inputs.

The mixed-precision solver stores, for every output site n of parity p, the 16
matrices that multiply its neighbours (the terms of Eq. (5) plus the three-hop
terms, with eta, the boundary sign and c_N folded in), in the order
    k = 4 mu + 0 : eta_mu(n) s(n,1) F_mu(n)                  neighbour n + mu
    k = 4 mu + 1 : -eta_mu(n) s(n-mu,1) F_mu(n-mu)^dag       neighbour n - mu
    k = 4 mu + 2 : c_N eta_mu(n) s(n,3) W_mu(n)              neighbour n + 3mu
    k = 4 mu + 3 : -c_N eta_mu(n) s(n-3mu,3) W_mu(n-3mu)^dag neighbour n - 3mu
and rounds them to binary32, or to binary16 with one binary32 scale per site for
the eight one-hop matrices and one for the eight three-hop matrices.  Colour
vectors are rounded per site (quant.py).  The functions here build those
matrices from the definition, round them with the rules of quant.py, and apply
them in FP64, so that the GPU's FP32 arithmetic can be bounded against them.
"""
from __future__ import annotations

import numpy as np

from . import quant
from .geometry import eta as eta_field, parity

NAIK_COEFF = -1.0 / 24.0


def output_sites(dims, out_parity: int, cbs=None):
    """Coordinates [S][4] (x, y, z, t) of the output sites: all sites of parity out_parity in checkerboard
    order (cbs None), or the sites with checkerboard indices cbs, cb = (x + Lx (y + Ly (z + Lz t))) / 2."""
    Lx, Ly, Lz, Lt = dims
    if cbs is None:
        t, z, y, x = np.nonzero(parity(dims) == out_parity)   # lexicographic order = cb order
        return np.stack([x, y, z, t], axis=1)
    cbs = np.asarray(cbs, dtype=np.int64)
    rest = cbs // (Lx // 2)
    y = rest % Ly
    z = (rest // Ly) % Lz
    t = rest // (Ly * Lz)
    x = 2 * (cbs % (Lx // 2)) + (y + z + t + out_parity) % 2
    return np.stack([x, y, z, t], axis=1)


def site_matrices(fat, lng, dims, out_parity: int, antiperiodic_t: bool = True, naik: float = NAIK_COEFF,
                  cbs=None):
    """Return (mats [S][16][3][3], nbr [S][16]) for the output sites of parity out_parity: all V/2 of them,
    or the checkerboard indices cbs (see output_sites)."""
    Lx, Ly, Lz, Lt = dims
    L = np.array(dims)
    n = output_sites(dims, out_parity, cbs)
    x, y, z, t = n.T
    half = len(x)
    mats = np.zeros((half, 16, 3, 3), dtype=np.complex128)
    nbr = np.zeros((half, 16), dtype=np.int64)

    def cb(m):
        return (m[:, 0] + Lx * (m[:, 1] + Ly * (m[:, 2] + Lz * m[:, 3]))) // 2

    def sign(mu, k, m):
        if mu != 3 or not antiperiodic_t:
            return np.ones(len(m))
        return np.where(((m[:, 3] + k) // Lt) % 2 == 0, 1.0, -1.0)

    for mu in range(4):
        e = eta_field(mu, dims)[t, z, y, x]
        for j, (k, U, c) in enumerate(((1, fat, 1.0), (3, lng, naik))):
            fwd = n.copy()
            fwd[:, mu] = (n[:, mu] + k) % L[mu]
            bwd = n.copy()
            bwd[:, mu] = (n[:, mu] - k) % L[mu]
            nbr[:, 4 * mu + 2 * j] = cb(fwd)
            nbr[:, 4 * mu + 2 * j + 1] = cb(bwd)
            if U is None:
                continue
            Uf = U[mu, n[:, 3], n[:, 2], n[:, 1], n[:, 0]]
            Ub = U[mu, bwd[:, 3], bwd[:, 2], bwd[:, 1], bwd[:, 0]]
            mats[:, 4 * mu + 2 * j] = (c * e * sign(mu, k, n))[:, None, None] * Uf
            mats[:, 4 * mu + 2 * j + 1] = (-c * e * sign(mu, k, bwd))[:, None, None] * np.conj(
                np.swapaxes(Ub, -1, -2))
    return mats, nbr


def folded_scalars(dims, out_parity: int, antiperiodic_t: bool = True, naik: float = NAIK_COEFF, cbs=None):
    """The real scalar folded into each of the 16 matrices of site_matrices: [S][16]
    (eta_mu(n) s(start, k), times c_N for three-hop matrices and -1 for backward ones)."""
    Lx, Ly, Lz, Lt = dims
    n = output_sites(dims, out_parity, cbs)
    x, y, z, t = n.T
    out = np.zeros((len(x), 16))
    for mu in range(4):
        e = eta_field(mu, dims)[t, z, y, x]
        for j, (k, c) in enumerate(((1, 1.0), (3, naik))):
            bwd = n.copy()
            bwd[:, mu] = (n[:, mu] - k) % dims[mu]
            for d, start, sgn in ((0, n, 1.0), (1, bwd, -1.0)):
                s = np.ones(len(x))
                if mu == 3 and antiperiodic_t:
                    s = np.where(((start[:, 3] + k) // Lt) % 2 == 0, 1.0, -1.0)
                out[:, 4 * mu + 2 * j + d] = sgn * c * e * s
    return out


def rebuild_third_rows(mats, scalars, ks):
    """For matrices s U with U in SU(3), replace row 3 by (a' x b')^* / s from rows 1 and 2 (paper Sec. 3.3)."""
    out = mats.copy()
    for k in ks:
        a, b = mats[:, k, 0], mats[:, k, 1]
        out[:, k, 2] = np.conj(np.cross(a, b)) / scalars[:, k, None]
    return out


def apply_site_matrices(mats, nbr, chi_half):
    """out(n) = sum_k mats[n,k] chi(nbr[n,k]) in FP64."""
    return np.einsum("nkab,nkb->na", mats, chi_half[nbr])


def abs_bound_terms(mats, nbr, chi_half):
    """sum_k |mats[n,k]| |chi(nbr[n,k])| per output component (for rounding-error bounds)."""
    return np.einsum("nkab,nkb->na", np.abs(mats.real) + np.abs(mats.imag),
                     np.abs(chi_half[nbr].real) + np.abs(chi_half[nbr].imag))


K_FAT = [4 * mu + d for mu in range(4) for d in (0, 1)]
K_LONG = [4 * mu + d for mu in range(4) for d in (2, 3)]


def round_matrices(mats, prec: str, long12: bool = False, scalars=None):
    """Round the 16 matrices of each site as the storage format does.

    long12: the three-hop matrices are stored as their first two rows (rounded like every stored
    value; FP16 scale over the stored entries only) and the third row is rebuilt from them with
    the folded scalars (see folded_scalars).
    """
    if prec == "f64":
        out = mats.copy()
    elif prec == "f32":
        out = quant.to_f32(mats)
    elif prec == "f16":
        out = np.empty_like(mats)
        codes, s = quant.quantize_link_group_f16(mats[:, K_FAT])
        out[:, K_FAT] = quant.dequantize_link_group_f16(codes, s)
        if long12:
            codes, s = quant.quantize_link_group_f16(mats[:, K_LONG][:, :, :2, :])
            out[:, K_LONG, :2, :] = quant.dequantize_link_group_f16(codes, s)
        else:
            codes, s = quant.quantize_link_group_f16(mats[:, K_LONG])
            out[:, K_LONG] = quant.dequantize_link_group_f16(codes, s)
    else:
        raise ValueError(prec)
    if long12:
        out = rebuild_third_rows(out, scalars, K_LONG)
    return out


def round_spinor(v, prec: str):
    if prec == "f64":
        return v
    if prec == "f32":
        return quant.to_f32(v)
    if prec == "f16":
        return quant.spinor_f16_roundtrip(v)
    raise ValueError(prec)
