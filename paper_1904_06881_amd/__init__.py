"""MI355X-native ternary high-density-ratio free-energy lattice Boltzmann
update with wetting walls (arXiv:1904.06881).

The compute path is the HIP library ``liblbm3.so`` behind the C ABI declared in
``include/lbm3.h``; :mod:`paper_1904_06881_amd.lbm3` is its ctypes binding.
Importing the package itself loads nothing; :mod:`.inputs` builds synthetic
initial fields.
"""
__all__ = ["inputs", "lbm3"]
