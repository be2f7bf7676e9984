"""ENO-AO (arXiv 2108.12742) on MI355X: HIP kernels for gfx950 behind a C ABI.

Submodules:
  enoao      ctypes binding of libenoao.so (include/enoao.h), same function names
  workloads  seeded synthetic initial data
  build      in-tree hipcc build of libenoao.so
"""
