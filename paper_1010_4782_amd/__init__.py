"""MI355X-native staggered-fermion CG: HIP kernels for gfx950 behind the C ABI of include/stagcg.h.

The solver computes x_e = (4 m^2 - D_eo D_oe)^{-1} b_e for the staggered Dirac
operator of Kim and Lee (Lattice 2010), Eq. (5) with folded phases, plus a
three-hop Naik term.  `paper_1010_4782_amd.stagcg` holds the torch-facing
binding; `paper_1010_4782_amd.build` compiles libstagcg.so.
"""

__all__ = ["Lattice", "cg_solve_batch", "StagError"]


def __getattr__(name):
    if name in __all__:
        from . import stagcg

        return getattr(stagcg, name)
    raise AttributeError(name)
