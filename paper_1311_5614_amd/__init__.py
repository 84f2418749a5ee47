"""MI355X-native implicit immersed-boundary multigrid solver (gfx950 HIP).

The compute path is libibmg.so (C ABI in include/ibmg.h); `ibmg` is its thin
ctypes binding.  Importing the binding raises if the library is not built.
"""
__all__ = ["ibmg", "build"]
