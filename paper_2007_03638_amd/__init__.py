"""MI355X (gfx950) implementation of Riemannian optimisation of an infinite binary MERA.

The compute path is the HIP library libmera_hip.so (C ABI in include/mera.h); `api` is its Python binding.
Importing this package loads nothing; the first API call loads the library and fails if it is not built.
"""
__all__ = ["api", "inputs", "build"]
