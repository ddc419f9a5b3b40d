"""MI355X (gfx950) hot path of adjoint-based optimal control for a coupled
anisotropic chemotaxis system with MRT / AMRT lattice Boltzmann models
(arXiv:1908.03876).

Submodules:
  inputs  - seeded synthetic workloads (no method arithmetic)
  abi     - ctypes binding of the C-ABI in include/mrt.h (libmrt.so)
  solver  - device-resident problems, tapes, the gradient iteration
  build   - hipcc build of libmrt.so for gfx950
"""
