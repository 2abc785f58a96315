"""MI355X (gfx950) implementation of the 3rd-order recursive-filter horizontal
covariance operator V_H = G_y G_x of Farina et al. (arXiv:1404.5756).

Submodules:
  rf3       -- ctypes binding of the C ABI in include/rf3.h (librf3.so)
  operator  -- HorizontalCovariance (grid + coefficient block: apply, adjoint,
               one direction, the plain and the fused 1st-RF) and Batch
  var3d     -- RF3XY (torch.autograd.Function), Observations, Var3D (cost,
               gradient, conjugate gradients) and the synthetic 3D-VAR problem
  synth     -- seeded synthetic workloads
  build     -- hipcc build of librf3.so

Importing the package loads nothing; librf3.so is loaded on first use.
"""
__all__ = ["rf3", "operator", "var3d", "synth", "build"]
