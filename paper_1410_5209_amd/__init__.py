"""MI355X (gfx950) implementation of the SALS / CDTF row-update path of
Shin & Kang, "Distributed Methods for High-dimensional and Large-scale Tensor
Factorization" (arXiv:1410.5209), behind the C ABI of include/tf.h.

The computation lives in the HIP library ``libtfsals.so``; ``tf`` is its thin
ctypes binding and ``model`` a convenience wrapper that owns the device
buffers (torch supplies device memory and streams only).
"""
from . import tf  # noqa: F401
