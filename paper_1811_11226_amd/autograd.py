"""torch.autograd.Function wrappers of the differentiable warps.

The forward calls run the library's fused warp, by default with photometrics
disabled (intensity out = interpolated value, fill outside).  The affine warp
also takes a photometric parameter set without window: gain, offset, noise
and occlusion are affine in the interpolated value V (out = gain V + offset
+ sigma n, with V = 0 on the occluded slab), so the adjoint receives
gain * grad_out, zero on the slab.  The backward calls run the library's
adjoint kernels.  M (12 values, [A|b] row-major) may live on the CPU or the
GPU; its gradient is returned on the same device, in M's dtype.
"""
import numpy as np
import torch

from . import ops


def _m_host(M):
    return M.detach().to("cpu", torch.float64).numpy()


def _photo_scale(grad_out, photo):
    """gain * grad_out, zero on the occluded slab (float32 gain, as the kernel)."""
    if photo is None:
        return grad_out
    if getattr(photo, "window", False):
        raise ValueError("the windowed photometric chain is not differentiated; pass window=False")
    g = grad_out * float(np.float32(photo.gain))
    if getattr(photo, "occlude", False):
        z = torch.arange(g.shape[2], device=g.device, dtype=torch.float32)
        lo, hi = float(np.float32(photo.occ_lo)), float(np.float32(photo.occ_hi))
        g = g * ((z < lo) | (z > hi)).to(g.dtype)
    return g


class WarpAffineFn(torch.autograd.Function):
    """out = warp(img; M) (then gain/offset/noise/occlusion when photo is given,
    without window) with gradients to img (scatter-add adjoint) and M."""

    @staticmethod
    def forward(ctx, img, M, fill=-1000.0, out_dim=None, photo=None):
        if photo is not None and getattr(photo, "window", False):
            raise ValueError("the windowed photometric chain is not differentiated")
        Mh = _m_host(M)
        out, _ = ops.warp_affine(img, Mh, fill=fill, out_dim=out_dim, photo=photo)
        ctx.save_for_backward(img)
        ctx.Mh, ctx.fill, ctx.M_meta, ctx.photo = Mh, fill, (M.device, M.dtype), photo
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (img,) = ctx.saved_tensors
        g = _photo_scale(grad_out, ctx.photo).contiguous()
        g_img, g_M = ops.warp_affine_backward(img, ctx.Mh, g, fill=ctx.fill,
                                              want_img=ctx.needs_input_grad[0],
                                              want_M=ctx.needs_input_grad[1])
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, None, None, None


class WarpDisplacementFn(torch.autograd.Function):
    """out = warp(img; M, disp) with gradients to img, M and disp."""

    @staticmethod
    def forward(ctx, img, M, disp, fill=-1000.0):
        Mh = _m_host(M)
        out, _ = ops.warp_displacement(img, Mh, disp.contiguous(), fill=fill)
        ctx.save_for_backward(img, disp)
        ctx.Mh, ctx.fill, ctx.M_meta = Mh, fill, (M.device, M.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, disp = ctx.saved_tensors
        g_img, g_M, g_disp = ops.warp_displacement_backward(
            img, ctx.Mh, disp.contiguous(), grad_out.contiguous(), fill=ctx.fill,
            want_img=ctx.needs_input_grad[0], want_M=ctx.needs_input_grad[1],
            want_disp=ctx.needs_input_grad[2])
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, g_disp, None


class WarpBsplineFn(torch.autograd.Function):
    """out = warp(img; M, B ctrl) with the B-spline displacement evaluated in
    the warp kernel; gradients to img, M and the control grid ctrl."""

    @staticmethod
    def forward(ctx, img, M, ctrl, fill=-1000.0, out_dim=None):
        Mh = _m_host(M)
        out, _ = ops.warp_bspline(img, Mh, ctrl.contiguous(), fill=fill, out_dim=out_dim)
        ctx.save_for_backward(img, ctrl)
        ctx.Mh, ctx.fill, ctx.M_meta = Mh, fill, (M.device, M.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, ctrl = ctx.saved_tensors
        g_img, g_M, g_ctrl = ops.warp_bspline_backward(
            img, ctx.Mh, ctrl.contiguous(), grad_out.contiguous(), fill=ctx.fill,
            want_img=ctx.needs_input_grad[0], want_M=ctx.needs_input_grad[1],
            want_ctrl=ctx.needs_input_grad[2])
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, g_ctrl, None, None


class BSplineUpsampleFn(torch.autograd.Function):
    """disp = B ctrl (cubic B-spline upsampling) with gradient B^T g."""

    @staticmethod
    def forward(ctx, ctrl, out_dim):
        ctx.grid = tuple(ctrl.shape[1:])
        return ops.bspline_upsample(ctrl.contiguous(), out_dim)

    @staticmethod
    def backward(ctx, grad_disp):
        return ops.bspline_upsample_adjoint(grad_disp.contiguous(), ctx.grid), None


def warp_affine(img, M, fill=-1000.0, out_dim=None, photo=None):
    return WarpAffineFn.apply(img, M, fill, out_dim, photo)


def warp_displacement(img, M, disp, fill=-1000.0):
    return WarpDisplacementFn.apply(img, M, disp, fill)


def warp_bspline(img, M, ctrl, fill=-1000.0, out_dim=None):
    return WarpBsplineFn.apply(img, M, ctrl, fill, out_dim)


def bspline_upsample(ctrl, out_dim):
    return BSplineUpsampleFn.apply(ctrl, out_dim)
