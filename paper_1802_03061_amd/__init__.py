"""MI355X-native homogeneous-medium solver for the angularly reduced radiative transfer equation.

The compute path lives in the HIP library ``librte.so`` built from ``csrc/``; ``rte`` is a thin
ctypes binding to its C ABI (``include/rte.h``).  Importing this package does not load the
library: ``from paper_1802_03061_amd import rte`` does, and fails loudly if it is not built.
"""
__all__ = ["inputs", "rte"]
