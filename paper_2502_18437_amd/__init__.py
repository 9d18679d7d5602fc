"""MI355X-native explicit MLS-MPM substep (CRESSim-MPM, arXiv 2502.18437).

* ``paper_2502_18437_amd.mpm``: ctypes binding of the C ABI (include/mpm.h)
  to the HIP library ``libmpm.so`` (importing it requires the built library).
* ``paper_2502_18437_amd.scenes``: seeded synthetic input generators.
* ``paper_2502_18437_amd.build``: hipcc build of the library for gfx950.
"""
