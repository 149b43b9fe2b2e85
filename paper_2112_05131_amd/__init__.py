"""Plenoxels hot path (arXiv 2112.05131) on MI355X: a C-ABI HIP library
(include/plenoxel.h, csrc/) with a thin Python binding.

Submodules:
  binding   ctypes wrappers with the C function names (plx_*)
  grid      Grid container (index, records, occupancy, FP32 master)
  autograd  RenderFn / render(): torch.autograd over plx_render_fwd/bwd
  train     Trainer: fused render+MSE+backward, TV, sparse RMSProp
  build     hipcc build of the library
"""
from . import binding  # noqa: F401
