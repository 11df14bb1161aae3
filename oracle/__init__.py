"""CPU reference (oracle) of the finite-difference lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 restatement of
the scheme of Pan, Xu, Zhang & Jiang, "Lattice Boltzmann approach to high-speed
compressible flows" (2007): the Kataoka-Tsutahara D2V9 discrete-velocity model
(Sec. 2, Eqs. (e14)-(e18)), the forward-Euler / beta-mixed upwind finite
difference scheme (Eqs. (SEC-VON-1), (SEC-VON-2a/2b)) with the added dissipation
term (Eqs. (SEC-VON-11), (SEC-VON-13)), and the von Neumann amplification matrix
(Eqs. (SEC-VON-8), (SEC-VON-9), (SEC-VON-12)).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it. The GPU library never calls it, and it shares no code with the GPU
library: the two meet only in the seeded input generators of `workloads`.

Arithmetic is plain PyTorch on the CPU in float64 (so autograd can tape a
reference gradient); no blocking, fusion or reordering beyond the formulas.
"""
from . import kt, scheme, vonneumann  # noqa: F401
