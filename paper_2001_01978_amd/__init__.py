"""MI355X-native exact diagonalisation of general pairing Hamiltonians.

The compute path is the HIP library libpairdiag.so (built from csrc/ by
build.py) behind the C ABI declared in include/pairdiag.h; `pairdiag` is its
thin ctypes binding.  Importing this package loads nothing; the library is
loaded on first use of `pairdiag` and its absence is an error.
"""
