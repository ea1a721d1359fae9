"""MI355X-native DAFMM + HODLR-preconditioned GMRES for the 2D Lippmann-Schwinger equation.

The compute path lives in the HIP/C++ library ``libls.so`` (built from ``csrc/``);
``paper_2204_00326_amd.ls`` is its thin ctypes binding.  ``inputs`` holds the
seeded synthetic problem generators.  Importing this package loads nothing native.
"""
__all__ = ["inputs", "ls"]
