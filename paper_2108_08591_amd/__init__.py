"""MI355X-native MDF-LBM: the hot path of the multiple-distribution-function
MRT lattice Boltzmann method (Chai, Shi & Zhan, arXiv 2108.08591) as HIP
kernels for gfx950 behind a C ABI (``include/mdf.h``).

Importing the package loads nothing; ``paper_2108_08591_amd.mdf`` loads the
native library on first use and fails loudly if it is missing.
"""
__all__ = ["cases", "mdf"]
