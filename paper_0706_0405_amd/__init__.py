"""MI355X (gfx950) finite-difference lattice Boltzmann step on the KT D2V9 model.

Pan, Xu, Zhang & Jiang, "Lattice Boltzmann approach to high-speed compressible
flows" (2007): the D2V9 discrete-velocity model (Sec. 2), the beta-mixed upwind
finite-difference step with the added dissipation term (Secs. 2-3). The step
runs in hand-written HIP kernels (liblbkt.so, C ABI in include/lbkt.h); this
package is the thin Python binding over torch device tensors.
"""
from . import _lib  # noqa: F401
from .api import (Batch, Grid, autotune, check_flags, empty, init, init_adjoint, interior, invariants, moments,  # noqa: F401
                  run, step, step_adjoint, validate)
