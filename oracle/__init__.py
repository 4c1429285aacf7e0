"""CPU FP64 correctness oracle for the AARMR analysis step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library; both sides read their inputs from :mod:`synth`, which holds no
arithmetic of the method.

Everything here is plain and slow on purpose: an assembled sparse global
stiffness matrix, a direct Cholesky solve, explicit filter matrices, and the
combined-approximation and multigrid steps in the order and notation of the
paper (Yin, Wang, Li, Guo, "An efficient topology optimization method based
on adaptive reanalysis with projection reduction", arXiv 2205.00385).

Layout: the oracle stores vectors node-interleaved (AoS): global DOF
``3 * node + c``.  Node ``(i, j, k)`` has index ``i + (nx+1) * (j + (ny+1) * k)``
and element ``(i, j, k)`` has index ``i + nx * (j + ny * k)``.
"""

from . import fem, solve, sens, filt, mg, ca, oc  # noqa: F401
