"""Voronoi particle merging (Luu, Tueckmantel, Pukhov) as a HIP library for AMD Instinct MI355X.

Submodules:
  vpm        ctypes binding of libvpm.so (include/vpm.h); all arithmetic runs in HIP kernels
  workloads  seeded synthetic particle populations
  build      hipcc build of libvpm.so for gfx950
"""
__all__ = ["vpm", "workloads", "build"]
