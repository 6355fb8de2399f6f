"""MI355X FFA periodicity search: HIP kernels for gfx950 behind a C ABI.

Submodules:
  ffa    -- ctypes binding of libffa.so (plans, search, fold, batch, server)
  synth  -- seeded synthetic inputs (no search arithmetic)
  build  -- hipcc build of libffa.so
"""
