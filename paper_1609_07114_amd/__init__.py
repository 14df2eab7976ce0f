"""MI355X (gfx950) library for the stable FDTD method with embedded
reduced-order models.

  capi        ctypes binding of include/fdtd_rom.h (same entry-point names)
  sim         Simulation: PyTorch device workspace + stream, HIP compute
  build       in-tree hipcc build of libfdtdrom.so
"""
