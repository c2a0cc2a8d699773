"""MI355X-native Hartree step of the LASTO method (Kang, Davenport, Glimm,
Keyes, McGuigan, "Linear Augmented Slater-Type Orbital Method for Free
Standing Clusters").

The compute path lives in ``csrc/`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/lasto.h``); ``lasto`` is the thin ctypes binding.
``inputs`` holds the seeded synthetic workload generators only.

Importing the package loads nothing native; ``paper_0806_1723_amd.lasto``
loads ``liblasto.so`` and raises if it has not been built.
"""

__all__ = ["inputs", "lasto"]
