"""Randomized generalized SVD of matrix pairs on AMD MI355X (gfx950).

The computation lives in the HIP library librgsvd.so (C ABI, include/rgsvd.h);
``rgsvd`` is its ctypes binding.  Importing the package loads nothing; the
library is loaded on first use and an unbuilt library raises.
"""
__all__ = ["rgsvd", "inputs", "build"]
