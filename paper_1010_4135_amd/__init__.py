"""MI355X-native 3D finite-difference lattice Boltzmann solver (Chen, Xu,
Zhang and Li, arXiv:1010.4135): the 15-velocity Kataoka-Tsutahara model with
NND convection, artificial dissipation and BGK relaxation, advanced by a fused
HIP kernel for gfx950 behind the C-ABI library declared in include/lbm3d.h.

Submodules:
  lbm3d    -- ctypes binding of the C-ABI (loads the in-tree HIP library and
              fails loudly if it is missing)
  inputs   -- seeded synthetic workloads (initial fields, run parameters)
  metrics  -- error norms used to compare solutions
"""
