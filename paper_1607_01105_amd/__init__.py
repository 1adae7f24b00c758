"""MI355X-native hot path of the operator-splitting PPML scheme
(Kulikov & Vorobyov, arXiv:1607.01105).

The solver lives in the HIP library ``csrc/libppml.so`` behind the C ABI of
``include/ppml.h``; :mod:`paper_1607_01105_amd.ppml` is its ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
