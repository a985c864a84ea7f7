"""MI355X-native periodic DMET embedding transform (bath, one-body, ERIs).

The compute path is libdmet.so (hand-written HIP kernels for gfx950) behind
a C ABI declared in include/dmet.h; ``paper_1909_08596_amd.dmet`` is its thin
ctypes binding.  Importing this package does not load the library.
"""

__all__ = ["dmet"]
