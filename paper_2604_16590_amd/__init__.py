"""MI355X-native kernelised linear global attention.

The attention runs in hand-written gfx950 HIP kernels behind the C ABI of
liblinattn.so (include/la.h); this package is its Python binding.
"""
from ._binding import (LaError, LinearAttention, Plan, apply, apply_gated,  # noqa: F401
                       backward, forward, forward_gated, forward_noalloc, gen_fill, lib, linear_attention,
                       profile_enable, profile_read, stream_probe, tile_blend, tile_extract,
                       tile_geometry, tiled_attention, tiled_forward, workspace_size)

__all__ = ["forward", "forward_noalloc", "apply", "backward", "forward_gated", "apply_gated", "LinearAttention",
           "linear_attention", "gen_fill", "workspace_size", "lib", "LaError", "Plan",
           "profile_enable", "profile_read", "tile_extract", "tile_blend", "tile_geometry",
           "tiled_attention", "tiled_forward", "stream_probe"]
