"""Chemical-potential multiphase lattice Boltzmann (arXiv:1906.09530) on
AMD Instinct MI355X (gfx950).

The solver lives in the shared library ``libcplbm.so`` (HIP kernels behind a
C ABI, declared in ``include/lbm.h``); ``paper_1906_09530_amd.lbm`` is a thin
ctypes binding with the same entry-point names.  Importing this package does
not load the library; ``lbm.load()`` does, and raises if it is not built.
"""
