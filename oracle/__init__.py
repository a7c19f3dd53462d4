"""Plain FP64 CPU oracle for the staggered-fermion CG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The GPU library never calls it
and shares no code with it; the two meet only in the seeded input generators of
``stag_inputs``.

Everything here is complex128 NumPy written for a reader to check against the
paper (Kim and Lee, "Multi GPU Performance of Conjugate Gradient Algorithm with
Staggered Fermions", Lattice 2010):

  * geometry  - site coordinates, parity, staggered phases, boundary signs
  * dslash    - the staggered Dirac operator of Eq. (5) with the phases of
                Sec. 2 folded in and a three-hop (Naik) term added; even-odd
                blocks; the normal operator 4m^2 - D_eo D_oe; one-site evaluation
  * dense     - the same operator built as a dense matrix by scalar loops
  * free      - closed forms for unit links (plane-wave spectrum, FFT solve)
  * cg        - the conjugate-gradient loop of Fig. 1 with a true-residual check
  * fcg       - flexible CG with a preconditioner callback and stall fallback
  * quant     - FP32 / FP16-with-per-site-scale storage rules
  * lowprec   - the operator applied in FP64 to inputs rounded as the storage formats round them
  * cost      - bytes and flops per site (Sec. 2 accounting)
  * net       - the gauge-covariant linear network used as a preconditioner
  * fatten    - fat (one-hop) and long (three-hop) links built from a thin gauge
                field by explicit path products (the published asqtad recipe)

Readings of the paper where it is silent are stated in each function.
"""
from . import geometry, dslash, dense, free, cg, fcg, quant, cost, lowprec, net, fatten  # noqa: F401
