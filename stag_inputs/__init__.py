"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and the oracle.

This module only draws random numbers and shapes them into gauge links and
sources.  It holds none of the solver's arithmetic: no phases, no boundary
signs, no Dirac operator.  Both sides of every parity check consume the arrays
made here.

Layouts (the user layouts of the C ABI):
  * links  : complex128 [4][Lt][Lz][Ly][Lx][3][3]; index 0 of the first axis is
             the x direction, 3 is time.  Entry [mu][t][z][y][x] is the link
             U_mu(n) that carries colour from site n+mu to site n.
  * sources: complex128 [nrhs][V/2][3] on the even sites, site index
             cb = lex >> 1 with lex = x + Lx*(y + Ly*(z + Lz*t)).

Recipe (the synthetic stand-in for the paper's MILC 28^3x96 ensemble, which is
not available here):
  * su3(eps): exp(i eps H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0,1) and
    lambda_a the Gell-Mann matrices; eps = 0.3.  The exponential is taken with
    torch.linalg.matrix_exp on the CPU in complex128.
  * "unitary" links: su3(0.3).
  * "fat" links: 0.6 * su3(0.3) + 0.05 * (N(0,1) + i N(0,1)) per entry, which is
    not unitary.
  * sources: real and imaginary parts N(0,1) per colour component.
  * Generator: numpy PCG64 default_rng(seed).  Seeds for workload i (1-based):
    fat = 1000 i + 1, long = 1000 i + 2, source j = 1000 i + 10 + j.
  * The 48^3x144 link fields (two fields of 63.7M matrices, minutes on the host)
    follow the same recipe but are drawn on the GPU with a seeded torch generator
    (`random_su3_field_device`, `fat_field_device`, `workload_links_device`); the
    oracle reads host copies of those very tensors.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "GELL_MANN", "WORKLOADS", "su3_near_identity", "random_su3_field",
    "fat_field", "gaussian_source", "gaussian_source_device", "gaussian_full_field", "random_gauge_transform",
    "workload", "workload_links", "workload_sources", "point_sources", "half_volume", "volume",
    "random_su3_field_device", "fat_field_device", "workload_links_device", "DEVICE_LINK_WORKLOADS",
]


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


GELL_MANN = _gell_mann()

# Workloads: dims are (Lx, Ly, Lz, Lt); every run is antiperiodic in time.
WORKLOADS = {
    1: dict(name="8^4 plain FP64", lattices=[((8, 8, 8, 8), 1)], masses=[0.05],
            fat="unitary", tol=1e-10),
    2: dict(name="28^3x96 single RHS", lattices=[((28, 28, 28, 96), 1)], masses=[0.0062],
            fat="fat", tol=1e-10, reliable_interval=50),
    3: dict(name="batched 16^4x4 + 24^3x48x12 + 32^3x64x8",
            lattices=[((16, 16, 16, 16), 4), ((24, 24, 24, 48), 12), ((32, 32, 32, 64), 8)],
            masses=[0.01, 0.02, 0.05], fat="fat", tol=1e-10),
    4: dict(name="24^3x48 learned preconditioner", lattices=[((24, 24, 24, 48), 1)],
            masses=[0.01], fat="fat", tol=1e-10, train_pairs=2000, layers=4, channels=8),
    5: dict(name="48^3x144 x 8 RHS", lattices=[((48, 48, 48, 144), 8)], masses=[0.0062],
            fat="fat", tol=1e-10),
    # point sources at four times (three colours each) on one gauge field: the propagators of a
    # spectrum calculation and their pion correlator
    6: dict(name="28^3x96 point-source propagators", lattices=[((28, 28, 28, 96), 12)], masses=[0.0062],
            fat="fat", tol=1e-10, reliable_interval=50,
            source_sites=[(0, 0, 0, 0), (0, 0, 0, 24), (0, 0, 0, 48), (0, 0, 0, 72)]),
}
NAIK_COEFF = -1.0 / 24.0


def volume(dims) -> int:
    return int(np.prod(dims))


def half_volume(dims) -> int:
    return volume(dims) // 2


def su3_near_identity(rng: np.random.Generator, n: int, eps: float = 0.3) -> np.ndarray:
    """n matrices exp(i eps H), H a Gaussian traceless Hermitian 3x3 (Gell-Mann basis)."""
    import torch

    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, GELL_MANN) * 0.5
    U = torch.linalg.matrix_exp(torch.from_numpy(1j * eps * H)).numpy()
    return np.ascontiguousarray(U)


def _check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"dims must be four even extents >= 2, got {dims}")
    return dims


def random_su3_field(dims, seed: int, eps: float = 0.3) -> np.ndarray:
    """Link field of independent su3(eps) matrices, layout [4][Lt][Lz][Ly][Lx][3][3].

    Drawn one (mu, t) slab at a time so that memory stays bounded; the stream of
    random numbers does not depend on how the caller uses the result.
    """
    Lx, Ly, Lz, Lt = _check_dims(dims)
    rng = np.random.default_rng(seed)
    out = np.empty((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    slab = Lz * Ly * Lx
    for mu in range(4):
        for t in range(Lt):
            out[mu, t] = su3_near_identity(rng, slab, eps).reshape(Lz, Ly, Lx, 3, 3)
    return out


def fat_field(dims, seed: int, scale: float = 0.6, sigma: float = 0.05) -> np.ndarray:
    """scale * su3(0.3) + sigma * (N + iN) per entry: a non-unitary 'fat' link field."""
    U = random_su3_field(dims, seed)
    rng = np.random.default_rng([seed, 1])
    U *= scale
    for mu in range(4):
        for t in range(U.shape[1]):
            shp = U[mu, t].shape
            U[mu, t] += sigma * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    return U


def gaussian_source(dims, seed: int, nrhs: int = 1) -> np.ndarray:
    """Even-site Gaussian sources, complex128 [nrhs][V/2][3]."""
    dims = _check_dims(dims)
    rng = np.random.default_rng(seed)
    shp = (nrhs, half_volume(dims), 3)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def gaussian_source_device(dims, seed: int, nrhs: int, device="cuda"):
    """Even-site Gaussian sources drawn on the GPU with a seeded torch generator, complex128
    [nrhs][V/2][3]: the bulk training sources of the learned preconditioner (thousands of fields,
    too many to draw on the host and copy).  Deterministic for a given seed, device type and
    torch version."""
    import torch

    dims = _check_dims(dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    shp = (nrhs, half_volume(dims), 3)
    re = torch.randn(shp, generator=g, dtype=torch.float64, device=device)
    im = torch.randn(shp, generator=g, dtype=torch.float64, device=device)
    return torch.complex(re, im)


def gaussian_full_field(dims, seed: int) -> np.ndarray:
    """Full-lattice Gaussian colour vector field, complex128 [Lt][Lz][Ly][Lx][3]."""
    Lx, Ly, Lz, Lt = _check_dims(dims)
    rng = np.random.default_rng(seed)
    shp = (Lt, Lz, Ly, Lx, 3)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """One su3(1.0) matrix per site, complex128 [Lt][Lz][Ly][Lx][3][3]."""
    Lx, Ly, Lz, Lt = _check_dims(dims)
    rng = np.random.default_rng(seed)
    g = su3_near_identity(rng, Lt * Lz * Ly * Lx, eps=1.0)
    return g.reshape(Lt, Lz, Ly, Lx, 3, 3)


def random_su3_field_device(dims, seed: int, eps: float = 0.3, device="cuda"):
    """The su3(eps) recipe of random_su3_field drawn on the GPU: a complex128 torch tensor
    [4][Lt][Lz][Ly][Lx][3][3] from a torch generator seeded with `seed`, eight time slices at a time.
    Deterministic for a given seed, device type and torch version (not the host stream)."""
    import torch

    Lx, Ly, Lz, Lt = _check_dims(dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    lam = torch.from_numpy(GELL_MANN.reshape(8, 9)).to(device)
    out = torch.empty((4, Lt, Lz, Ly, Lx, 3, 3), dtype=torch.complex128, device=device)
    slab = Lz * Ly * Lx
    for mu in range(4):
        for t0 in range(0, Lt, 8):
            n = min(8, Lt - t0)
            h = torch.randn((n * slab, 8), generator=g, dtype=torch.float64, device=device)
            H = (h.to(torch.complex128) @ lam).reshape(n * slab, 3, 3) * 0.5
            out[mu, t0:t0 + n] = torch.linalg.matrix_exp(1j * eps * H).reshape(n, Lz, Ly, Lx, 3, 3)
    return out


def fat_field_device(dims, seed: int, scale: float = 0.6, sigma: float = 0.05, device="cuda"):
    """fat_field's recipe on the GPU: scale * su3(0.3) + sigma * (N + iN) per entry, the noise from a
    second generator seeded with 1000003 * seed + 1."""
    import torch

    U = random_su3_field_device(dims, seed, device=device)
    U *= scale
    g = torch.Generator(device=device)
    g.manual_seed(1000003 * int(seed) + 1)
    for mu in range(4):
        for t in range(U.shape[1]):
            shp = U[mu, t].shape
            re = torch.randn(shp, generator=g, dtype=torch.float64, device=device)
            im = torch.randn(shp, generator=g, dtype=torch.float64, device=device)
            U[mu, t] += sigma * torch.complex(re, im)
    return U


# workloads whose link fields are drawn on the GPU (their host generation takes minutes)
DEVICE_LINK_WORKLOADS = (5,)


def workload_links_device(i: int, lattice_index: int = 0, device="cuda"):
    """(fat, long) of workload i as torch tensors on the GPU: drawn there for the workloads in
    DEVICE_LINK_WORKLOADS, otherwise the host fields of workload_links copied over."""
    import torch

    w = WORKLOADS[i]
    if i not in DEVICE_LINK_WORKLOADS:
        fat, lng = workload_links(i, lattice_index)
        return torch.from_numpy(fat).to(device), torch.from_numpy(lng).to(device)
    dims = w["lattices"][lattice_index][0]
    seed_f = 1000 * i + 1 + 100 * lattice_index
    seed_l = 1000 * i + 2 + 100 * lattice_index
    fat = random_su3_field_device(dims, seed_f, device=device) if w["fat"] == "unitary" else \
        fat_field_device(dims, seed_f, device=device)
    return fat, random_su3_field_device(dims, seed_l, device=device)


def workload(i: int) -> dict:
    return WORKLOADS[i]


def workload_links(i: int, lattice_index: int = 0):
    """(fat, long) link fields of workload i for its lattice_index-th lattice."""
    w = WORKLOADS[i]
    dims = w["lattices"][lattice_index][0]
    seed_f = 1000 * i + 1 + 100 * lattice_index
    seed_l = 1000 * i + 2 + 100 * lattice_index
    fat = random_su3_field(dims, seed_f) if w["fat"] == "unitary" else fat_field(dims, seed_f)
    lng = random_su3_field(dims, seed_l)
    return fat, lng


def workload_sources(i: int, lattice_index: int = 0, nrhs: int | None = None) -> np.ndarray:
    w = WORKLOADS[i]
    dims, n = w["lattices"][lattice_index]
    if "source_sites" in w:
        return point_sources(dims, w["source_sites"])
    n = n if nrhs is None else nrhs
    return gaussian_source(dims, 1000 * i + 10 + 100 * lattice_index, n)


def point_sources(dims, sites) -> np.ndarray:
    """Unit sources delta_{n, site} delta_{a, c} for each even site in sites and colour c = 0, 1, 2:
    complex128 [3 * len(sites)][V/2][3] (even-odd index cb = lex >> 1)."""
    Lx, Ly, Lz, Lt = _check_dims(dims)
    out = np.zeros((3 * len(sites), half_volume(dims), 3), dtype=np.complex128)
    for s, (x, y, z, t) in enumerate(sites):
        if (x + y + z + t) % 2:
            raise ValueError(f"source site {(x, y, z, t)} is odd; the even-site solve needs an even source")
        cb = (x + Lx * (y + Ly * (z + Lz * t))) // 2
        for c in range(3):
            out[3 * s + c, cb, c] = 1.0
    return out
