"""MI355X-native D2Q9 two-phase lattice Boltzmann step (standard and
well-balanced LBE of Guo, arXiv:2012.11075) behind a C ABI.

The binding (``lbm``) is imported lazily so that ``inputs`` can be used
without loading the HIP library.
"""
__all__ = ["inputs", "lbm"]
