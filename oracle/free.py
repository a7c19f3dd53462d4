"""Closed forms for unit links (the free field).

With all links equal to the identity, D^2 is translation invariant: the cross
terms between different directions cancel because eta_mu(n + k nu) differs from
eta_mu(n) by (-1)^k exactly when nu < mu, and eta_mu(n)^2 = 1.  Each direction
then contributes nabla_mu^2 with

  nabla_mu chi(n) = chi(n+mu) - chi(n-mu) + c_N (chi(n+3mu) - chi(n-3mu)),

whose plane-wave eigenvalue is 2i (sin p_mu + c_N sin 3p_mu).  Hence

  -D^2 e^{ipn} = 4 sum_mu (sin p_mu + c_N sin 3 p_mu)^2 e^{ipn},

with p_mu = 2 pi k / L_mu, and p_t = pi (2k+1) / L_t when time is antiperiodic.
D^2 keeps parity, so on even-site vectors -D_eo D_oe has the same spectrum and
M = 4 m^2 - D_eo D_oe is diagonal in momentum space.  (The factor 4 comes from
Eq. (5) having no 1/2 in front of the differences.)
"""
from __future__ import annotations

import numpy as np

from .geometry import embed, restrict

NAIK_COEFF = -1.0 / 24.0


def momenta(dims, antiperiodic_t: bool = True):
    """Per-direction momentum grids p_mu (x, y, z, t), FFT ordering."""
    ps = []
    for mu, L in enumerate(dims):
        k = np.arange(L)
        shift = np.pi / L if (mu == 3 and antiperiodic_t) else 0.0
        ps.append(2 * np.pi * k / L + shift)
    return ps


def free_eigenvalue(p, naik: float = NAIK_COEFF) -> float:
    """Eigenvalue of -D^2 at momentum p = (p_x, p_y, p_z, p_t)."""
    return 4.0 * sum((np.sin(q) + naik * np.sin(3 * q)) ** 2 for q in p)


def free_spectrum(dims, antiperiodic_t: bool = True, naik: float = NAIK_COEFF) -> np.ndarray:
    """-D^2 eigenvalue on the [t][z][y][x] momentum grid used by free_solve."""
    px, py, pz, pt = momenta(dims, antiperiodic_t)
    T, Z, Y, X = np.meshgrid(pt, pz, py, px, indexing="ij")
    lam = np.zeros(T.shape)
    for q in (X, Y, Z, T):
        lam += (np.sin(q) + naik * np.sin(3 * q)) ** 2
    return 4.0 * lam


def plane_wave(dims, p, antiperiodic_t: bool = True) -> np.ndarray:
    """e^{i p.n} on the full lattice, shape [Lt][Lz][Ly][Lx]."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))


def free_solve(b_e: np.ndarray, dims, mass: float, antiperiodic_t: bool = True,
               naik: float = NAIK_COEFF) -> np.ndarray:
    """x_e = M^{-1} b_e for unit links, by FFT.

    The antiperiodic time direction is made periodic by the twist e^{-i pi t / L_t},
    so that the FFT's momenta 2 pi k / L_t become p_t - pi / L_t.
    """
    Lx, Ly, Lz, Lt = dims
    b = embed(b_e, dims, 0)
    t = np.arange(Lt).reshape(Lt, 1, 1, 1, 1)
    twist = np.exp(-1j * np.pi * t / Lt) if antiperiodic_t else np.ones_like(t, dtype=complex)
    B = np.fft.fftn(b * twist, axes=(0, 1, 2, 3))
    denom = 4.0 * mass * mass + free_spectrum(dims, antiperiodic_t, naik)
    x = np.fft.ifftn(B / denom[..., None], axes=(0, 1, 2, 3)) / twist
    return restrict(x, dims, 0)


def unit_links(dims) -> np.ndarray:
    Lx, Ly, Lz, Lt = dims
    U = np.zeros((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U
