"""MI355X-native Chebyshev-filtered subspace iteration (arXiv 1305.5120).

The solver lives in the gfx950 shared library ``libchfsi.so`` (HIP kernels
behind the C ABI of ``include/chfsi.h``); ``paper_1305_5120_amd.chfsi`` is
its Python binding.  Importing the package loads nothing; the binding loads
the library on first use and fails loudly if it is missing.
"""
