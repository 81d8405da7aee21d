"""MI355X-native pixel-detector correction and photon finding.

Submodules:
  pdc    -- ctypes binding of the C-ABI library libpdc.so (HIP, gfx950)
  synth  -- seeded synthetic frames and calibration planes
  build  -- compiles libpdc.so with hipcc for gfx950

Importing the package loads nothing; ``paper_1903_06838_amd.pdc`` opens the
shared library on first use.
"""
