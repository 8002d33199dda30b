"""MI355X (gfx950) implementation of the hot path of the multibody MFS scattering method.

The compute path is libmfs.so (HIP kernels behind a C ABI, include/mfs.h); ``mfs`` is its thin
Python binding and ``build`` compiles it in-tree.
"""

from . import mfs  # noqa: F401
