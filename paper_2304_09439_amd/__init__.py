"""LOCC crop-collision hot path for AMD MI355X (gfx950).

The compute lives in the HIP/C++ shared library ``liblocc.so`` built from
``csrc/``; :mod:`paper_2304_09439_amd.binding` is a thin ctypes layer over its
C-ABI (``include/locc.h``), and :mod:`paper_2304_09439_amd.inputs` draws the
seeded synthetic inputs.  Importing the package loads nothing; the library is
loaded on first use of the binding.
"""

__all__ = ["inputs", "binding"]
