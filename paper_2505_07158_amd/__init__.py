"""MI355X (gfx950) implementation of the diffusion-free per-frame video cipher
of arXiv 2505.07158: sub-frame SHA-256 frame hash, FP64 hyperchaotic-Lorenz
key schedule, and bit-level row/column circular shifts fused with one XOR
round, plus the exact inverse.

The compute path is the HIP library ``libvcipher.so`` (C ABI in
``include/vcipher.h``); ``paper_2505_07158_amd.vcipher`` is its ctypes
binding.  Build with ``python -m paper_2505_07158_amd.build``.
"""

__all__ = ["vcipher", "build"]
