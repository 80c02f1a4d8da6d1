"""MI355X-native CCPR-FDTD forward / adjoint / gradient library.

The compute path lives in the HIP/C++ shared library built from csrc/ (its
C-ABI is declared in include/ccprfdtd.h).  This package holds the thin ctypes
binding (``lib``, with the continuous-batching serving engine ``lib.Engine``),
workload set-up (``solver``), the density -> objective autograd functions
(``autograd``), a small optimisation loop (``topopt``) and the seeded
synthetic inputs (``inputs``).
Importing the package does not load the GPU library; ``lib.load()`` does, and
fails loudly when it has not been built.
"""

__all__ = ["inputs", "lib", "solver", "autograd", "topopt"]
