"""QUAPI tensor-propagator propagation of open-quantum-system density matrices on
AMD Instinct MI355X (gfx950).

Submodules:
  quapi      ctypes binding of the HIP library libquapi.so (C ABI in include/quapi.h)
  workloads  seeded synthetic inputs
  build      hipcc build of the library
  serve      continuous-batching server over the library
"""
__all__ = ["quapi", "workloads", "build"]
