"""MI355X (gfx950) library for the analysis step of AARMR topology
optimisation: matrix-free hex8 stiffness products, multigrid-preconditioned
CG, the PARM/CARM reduced model, compliance sensitivities and the density
filter, all in hand-written HIP kernels behind the C ABI of
``include/aarmr.h``.  :mod:`paper_2205_00385_amd.aarmr` is the Python binding.
"""

__all__ = ["aarmr", "build"]
