"""MI355X-native kernelised linear global attention.

The attention runs in hand-written gfx950 HIP kernels behind the C ABI of
liblinattn.so (include/la.h); this package is its Python binding.
"""
from ._binding import (LaError, LinearAttention, backward, forward, gen_fill,  # noqa: F401
                       lib, linear_attention, workspace_size)

__all__ = ["forward", "backward", "LinearAttention", "linear_attention", "gen_fill",
           "workspace_size", "lib", "LaError"]
