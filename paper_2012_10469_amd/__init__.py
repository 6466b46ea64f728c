"""MI355X-native low-rank Matrix Exponentiated Gradient (Garber & Kaplan,
arXiv 2012.10469): HIP kernels for gfx950 behind the C ABI of include/meg.h,
with a ctypes binding in ``paper_2012_10469_amd.meg``.

Importing the package does not load the library; ``paper_2012_10469_amd.meg``
does, and fails loudly when ``libmeg.so`` has not been built.
"""
__all__ = ["meg", "build"]
