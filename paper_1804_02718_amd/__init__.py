"""MI355X-native finite-difference integral fractional Laplacian (Duo & Zhang, arXiv:1804.02718).

The compute path lives in the HIP library ``libfl.so`` (built from ``csrc/``)
behind the C-ABI declared in ``include/fl.h``; ``paper_1804_02718_amd.fl`` is
its thin ctypes binding.  ``paper_1804_02718_amd.inputs`` holds the seeded
synthetic input generators.  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["fl", "inputs"]
