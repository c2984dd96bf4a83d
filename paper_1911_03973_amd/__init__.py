"""Element-based P1 finite-element solvers on MI355X (gfx950).

The compute path is the HIP library ``libfem.so`` behind the C ABI declared in
``include/fem.h``; :mod:`paper_1911_03973_amd.fem` is its thin ctypes binding.
Importing this package loads nothing; importing ``fem`` loads the library and
fails loudly if it has not been built.
"""
__all__ = ["inputs"]
