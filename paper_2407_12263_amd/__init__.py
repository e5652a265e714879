"""MI355X-native difference-free conservative phase-field lattice Boltzmann
solver (Zhao, Patel & Lee, arXiv 2407.12263).

The solver is the HIP library ``liblbm.so`` behind the C ABI of
``include/lbm.h``; :mod:`.lbm` is its thin Python binding and
:mod:`.inputs` builds the seeded synthetic workloads. Importing the package
loads nothing; the library is loaded on first use and a missing library is
an error, never a fallback.
"""
__all__ = ["lbm", "inputs"]
