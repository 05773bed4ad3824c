"""MI355X (gfx950) implementation of the positivity-preserving Lax-Wendroff discontinuous Galerkin
time step for the compressible Euler equations (Moe, Rossmanith, Seal, arXiv:1601.08145).

  lxw     -- the Python binding of the C interface in include/lxw.h (HIP library liblxw.so)
  inputs  -- seeded synthetic meshes and initial states
  build   -- in-tree build of liblxw.so with hipcc
"""
