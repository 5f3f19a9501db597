"""Seeded synthetic image pairs shaped like DeepMatching's workloads.

This package only draws and warps images; it contains none of the matching
method's arithmetic, so both the FP64 oracle and the GPU path can consume its
outputs without sharing any code of the method.
"""
from .pairs import (CONFIGS, CONFIG_NMAX, make_pair, sub_pair, make_batch, make_warp_pair, blurred_noise,
                    multi_octave_texture, smooth_field, warp_bilinear, shift_reflect, invert_field)

__all__ = ["CONFIGS", "CONFIG_NMAX", "make_pair", "sub_pair", "make_batch", "make_warp_pair", "blurred_noise",
           "multi_octave_texture", "smooth_field", "warp_bilinear", "shift_reflect", "invert_field"]
