"""MI355X (gfx950) CT data augmentation (Rister et al., arXiv:1811.11226).

C ABI: include/ctaug.h, implemented by libctaug.so (HIP kernels in csrc/).
Python: `ops` (one function per C entry point), `autograd` (differentiable
warps), `BatchPlan` (persistent batched launch with HIP graph and autotuner).
"""
from . import ops
from .ops import (BatchPlan, Pipeline, affine_matrix, autotune_cache_clear, autotune_cache_load,
                  autotune_cache_lookup, autotune_cache_save, box_muller, bspline_upsample,
                  bspline_upsample_adjoint, make_job, gaussian_smooth, noise, photometric_noise, resample_sigma, warp_affine,
                  warp_affine_backward, warp_bspline, warp_bspline_backward, warp_displacement, warp_displacement_backward,
                  warp_labels)
from ._lib import CtaugError, LIB_PATH

__all__ = ["ops", "BatchPlan", "Pipeline", "affine_matrix", "autotune_cache_clear",
           "autotune_cache_load", "autotune_cache_lookup", "autotune_cache_save", "box_muller", "bspline_upsample", "bspline_upsample_adjoint",
           "make_job", "noise", "photometric_noise", "warp_affine", "warp_affine_backward",
           "warp_bspline", "warp_bspline_backward", "warp_displacement", "warp_displacement_backward", "warp_labels", "gaussian_smooth",
           "resample_sigma", "CtaugError", "LIB_PATH"]
