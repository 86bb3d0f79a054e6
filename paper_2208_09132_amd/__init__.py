"""MI355X-native CDUGKS time-step library (gfx950 HIP kernels behind a C ABI).

Submodules:
  cdugks     -- ctypes binding of include/cdugks.h (loads libcdugks.so)
  workloads  -- seeded synthetic problems (initial moments only)
  build      -- hipcc build of libcdugks.so
"""
