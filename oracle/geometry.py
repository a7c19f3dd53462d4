"""Lattice geometry for the oracle.

Conventions (the paper fixes none of them; Sec. 2 only says the phases are
folded into the links):
  * dims = (Lx, Ly, Lz, Lt); direction mu = 0, 1, 2, 3 is x, y, z, t.
  * Full-lattice fields are NumPy arrays indexed [t][z][y][x]; direction mu
    lives on array axis 3 - mu.
  * Parity of n is (x + y + z + t) mod 2.  Even-odd vectors hold the sites of
    one parity in lexicographic order, which is the order cb = lex >> 1 with
    lex = x + Lx*(y + Ly*(z + Lz*t)) (Lx even).
  * Staggered phase eta_mu(n) = (-1)^(n_0 + ... + n_{mu-1}).
  * Boundary sign of a forward hop of length k from site n in direction mu:
    (-1)^floor((n_mu + k) / L_mu) when mu is time and the time direction is
    antiperiodic, otherwise 1.  It counts how often the hop wraps, which is
    what a twisted translation gives, also when L_t <= k.
"""
from __future__ import annotations

import numpy as np


def axis_of(mu: int) -> int:
    """Array axis of direction mu in a [t][z][y][x] field."""
    return 3 - mu


def coords(dims):
    """Integer coordinate arrays (x, y, z, t), each of shape [Lt][Lz][Ly][Lx]."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return x, y, z, t


def parity(dims) -> np.ndarray:
    x, y, z, t = coords(dims)
    return (x + y + z + t) % 2


def eta(mu: int, dims) -> np.ndarray:
    """Staggered phase eta_mu(n) = (-1)^(sum of the coordinates before mu)."""
    n = coords(dims)
    s = np.zeros_like(n[0])
    for nu in range(mu):
        s = s + n[nu]
    return np.where(s % 2 == 0, 1.0, -1.0)


def hop_sign(mu: int, k: int, dims, antiperiodic_t: bool) -> np.ndarray:
    """Boundary sign sigma_mu(n, k) of the forward hop n -> n + k mu, per start site n."""
    n_mu = coords(dims)[mu]
    if mu != 3 or not antiperiodic_t:
        return np.ones(n_mu.shape)
    wraps = (n_mu + k) // dims[mu]
    return np.where(wraps % 2 == 0, 1.0, -1.0)


def shift(field: np.ndarray, mu: int, k: int) -> np.ndarray:
    """(shift f)(n) = f(n + k mu) with periodic wrap, for k of either sign."""
    return np.roll(field, -k, axis=axis_of(mu))


def embed(v_half: np.ndarray, dims, par: int) -> np.ndarray:
    """Even-odd vector [V/2][3] of parity par -> full field [Lt][Lz][Ly][Lx][3], zero elsewhere."""
    Lx, Ly, Lz, Lt = dims
    full = np.zeros((Lt * Lz * Ly * Lx, 3), dtype=np.complex128)
    mask = parity(dims).reshape(-1) == par
    full[mask] = v_half
    return full.reshape(Lt, Lz, Ly, Lx, 3)


def restrict(full: np.ndarray, dims, par: int) -> np.ndarray:
    """Full field -> the [V/2][3] vector of its sites of parity par (lexicographic order)."""
    mask = parity(dims).reshape(-1) == par
    return full.reshape(-1, 3)[mask].copy()


def site_of_cb(cb: int, par: int, dims):
    """Coordinates (x, y, z, t) of the even-odd index cb of parity par."""
    Lx, Ly, Lz, Lt = dims
    xh = cb % (Lx // 2)
    rest = cb // (Lx // 2)
    y = rest % Ly
    rest //= Ly
    z = rest % Lz
    t = rest // Lz
    x = 2 * xh + ((y + z + t + par) % 2)
    return x, y, z, t


def cb_of_site(x, y, z, t, dims) -> int:
    Lx, Ly, Lz, Lt = dims
    return (x + Lx * (y + Ly * (z + Lz * t))) // 2
