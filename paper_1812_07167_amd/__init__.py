"""MI355X-native HPS direct solver for variable-coefficient Helmholtz impedance problems.

* ``paper_1812_07167_amd.hps``     ctypes binding of the C ABI in include/hps.h
* ``paper_1812_07167_amd.inputs``  seeded closed-form problem data (numpy only)
* ``paper_1812_07167_amd.build``   builds libhps.so with hipcc for gfx950

Importing the package loads nothing; the library is loaded on first use.
"""
