"""MI355X (gfx950) implementation of the 3rd-order recursive-filter horizontal
covariance operator V_H = G_y G_x of Farina et al. (arXiv:1404.5756).

Submodules:
  rf3       -- ctypes binding of the C ABI in include/rf3.h (librf3.so)
  operator  -- HorizontalCovariance: grid + coefficient block, apply/adjoint/rf1
  autograd  -- torch.autograd.Function and the synthetic 3D-VAR harness
  synth     -- seeded synthetic workloads
  build     -- hipcc build of librf3.so

Importing the package loads nothing; librf3.so is loaded on first use.
"""
__all__ = ["rf3", "operator", "synth", "build"]
