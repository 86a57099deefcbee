"""MI355X (gfx950) implementation of the parity-blocked rotated staggered Bloch
eigensolver: HIP kernels and solver drivers in libpbr.so (csrc/, C interface in
include/pbr.h) and a thin ctypes binding (pbr.py).  Importing this package loads
nothing; ``paper_2606_03599_amd.pbr.lib()`` loads the library and fails loudly if
it has not been built.
"""

__all__ = ["pbr", "build"]
