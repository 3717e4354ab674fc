"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This package only *draws* inputs: CT-like phantoms, raw random transform and
photometric parameters, upstream gradients and control grids.  It holds none
of the augmentation arithmetic (no coordinate maps, interpolation, noise
generation or matrix composition); both the GPU path and the oracle receive
these draws as inputs and compute everything else on their own.
"""
from .phantom import phantom, phantom_pair
from .draws import AugmentRanges, PhotoParams, draw_affine_params, draw_occlusion, draw_photo, \
    identity_affine_params, N_AFFINE_PARAMS
from . import configs

__all__ = ["phantom", "phantom_pair", "AugmentRanges", "PhotoParams", "draw_affine_params",
           "draw_occlusion", "draw_photo", "identity_affine_params", "N_AFFINE_PARAMS", "configs"]
