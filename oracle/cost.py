"""Bytes and flops of one Dslash per output site (paper Sec. 2 accounting).

Paper mode (Sec. 2): the one-hop operator in double precision, every link and
every neighbour read from memory once per use:
    flops = 8 matvecs x 72 = 576 (a complex 3x3 matrix-vector product counted
            as 36 complex multiply-adds, 2 flops each for real and imaginary)
    bytes = 8 links x 144 + 8 neighbours x 48 + 1 output x 48 = 1584.
The paper prints 576 flops and 1584 bytes per site, and 0.6 G flops and 1.6 GB
for the even sites of 28^3 x 96 (1.669e9 bytes, which is 1.55 GiB: the paper's
"giga" is binary).

Compulsory mode (used for the roofline): each link and the input field read
once, the output written once:
    B(prec, R) = 16 l + s_L + R (v_in + v_out),
with l, s_L, v the link, link-scale and colour-vector sizes of the storage
precision.  Flops of the asqtad operator: 16 matvecs of 66 flops (9 complex
multiplies at 6 and 6 complex adds at 2) plus 15 complex-vector additions of
6 flops = 1146 per site per right-hand side.
"""
from __future__ import annotations

LINK_BYTES = {"f64": 144, "f32": 72, "f16": 36}
LINK_SCALE_BYTES = {"f64": 0, "f32": 0, "f16": 8}
SPINOR_BYTES = {"f64": 48, "f32": 24, "f16": 16}   # f16: 12 B of codes + a 4 B scale


def paper_site_cost(naik: bool = False):
    """(flops, bytes) per output site with neighbours re-read (the paper's convention)."""
    nlinks = 16 if naik else 8
    return nlinks * 72, nlinks * 144 + nlinks * 48 + 48


def paper_even_sweep(dims, naik: bool = False):
    """(flops, bytes) of one Dslash over all even sites, paper convention."""
    f, b = paper_site_cost(naik)
    half = dims[0] * dims[1] * dims[2] * dims[3] // 2
    return f * half, b * half


def flops_per_site(naik: bool = True, nrhs: int = 1) -> int:
    nmat = 16 if naik else 8
    return nrhs * (nmat * 66 + (nmat - 1) * 6)


def compulsory_bytes_per_site(prec: str = "f64", nrhs: int = 1, naik: bool = True) -> int:
    nlinks = 16 if naik else 8
    s_l = LINK_SCALE_BYTES[prec] if naik else LINK_SCALE_BYTES[prec] // 2
    return nlinks * LINK_BYTES[prec] + s_l + nrhs * 2 * SPINOR_BYTES[prec]


def cg_iteration_bytes_per_site(prec: str = "f64") -> int:
    """Compulsory bytes per even site of one CG iteration as the GPU path runs it:
    Dslash(odd), Dslash(even) + xpay reading d, r -= alpha Ad (read r, Ad; write r),
    x += alpha d and d = r + beta d (read x, d, r; write x, d)."""
    v = SPINOR_BYTES[prec]
    xv = 24 if prec == "f16" else v          # the f16 solver keeps x in f32
    return (2 * compulsory_bytes_per_site(prec) + v
            + 3 * v + (2 * xv + 3 * v))
