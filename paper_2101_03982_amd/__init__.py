"""MI355X-native semi-Lagrangian off-lattice Boltzmann time step.

The time step of Wilde et al., "Cubature rules for weakly and fully
compressible off-lattice Boltzmann methods" (arXiv 2101.03982), Sec. 3, as
fused HIP kernels for gfx950 behind the C ABI of include/lbm.h (liblbm.so).
This package holds the build script, the HIP sources (csrc/) and a thin
Python binding; PyTorch supplies device memory and streams only.
"""
from .lattice import Diagnostics, Lattice, set_table, stencil  # noqa: F401
from .adjoint import KineticEnergyRollout, kinetic_energy_after, rollout_states  # noqa: F401

SETS = ("D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45")
