"""MI355X-native FFT-based pressure Poisson solver (FluTAS, arXiv 2204.08834, Section 3.3.1).

The solve runs in hand-written HIP kernels behind the C ABI declared in
``include/poisson.h`` (``libpoisson.so``); this package holds that library's
sources (``csrc/``), a thin ctypes binding (``poisson``), and the seeded
synthetic workloads (``inputs``).  Importing the package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""

__all__ = ["inputs", "poisson"]
