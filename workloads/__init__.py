"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Holds workload definitions (grids, parameters, boundary states, initial fields,
batched draws) and the gas-dynamics closed forms that define them. It contains
none of the lattice Boltzmann method's arithmetic.
"""
from . import gasdyn, problems  # noqa: F401
