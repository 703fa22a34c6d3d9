"""MI355X-native phaseless-AFQMC walker step (arXiv 2209.04015, ipie).

The compute path lives in the HIP/C++ shared library built from ``csrc/``
and exposed through the C ABI declared in ``include/afqmc.h``.  The Python
module :mod:`paper_2209_04015_amd.afqmc` is a thin ctypes binding over that
library (argument marshalling only).  :mod:`paper_2209_04015_amd.inputs`
holds the seeded synthetic input generators.
"""

__all__ = ["inputs", "afqmc"]
