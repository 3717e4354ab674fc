"""torch.autograd.Function wrappers of the differentiable warps.

The forward calls run the library's fused warp, by default with photometrics
disabled (intensity out = interpolated value, fill outside).  They also take
a photometric parameter set without window: gain, offset, noise and
occlusion are affine in the interpolated value, and the library's adjoint
calls apply their adjoint (gain, zero on the occluded slab) themselves; the
windowed chain is refused by the library.  M (12 values, [A|b] row-major)
may live on the CPU or the GPU; its gradient is returned on the same device,
in M's dtype.  Only argument marshalling happens here.
"""
import torch

from . import ops


def _m_host(M):
    return M.detach().to("cpu", torch.float64).numpy()


class WarpAffineFn(torch.autograd.Function):
    """out = warp(img; M) (then gain/offset/noise/occlusion when photo is given,
    without window) with gradients to img (scatter-add adjoint) and M."""

    @staticmethod
    def forward(ctx, img, M, fill=-1000.0, out_dim=None, photo=None):
        Mh = _m_host(M)
        out, _ = ops.warp_affine(img, Mh, fill=fill, out_dim=out_dim, photo=photo)
        ctx.save_for_backward(img)
        ctx.Mh, ctx.fill, ctx.M_meta, ctx.photo = Mh, fill, (M.device, M.dtype), photo
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (img,) = ctx.saved_tensors
        g_img, g_M = ops.warp_affine_backward(img, ctx.Mh, grad_out.contiguous(), fill=ctx.fill,
                                              want_img=ctx.needs_input_grad[0],
                                              want_M=ctx.needs_input_grad[1], photo=ctx.photo)
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, None, None, None


class WarpDisplacementFn(torch.autograd.Function):
    """out = warp(img; M, disp) (photometrics as WarpAffineFn) with gradients
    to img, M and disp."""

    @staticmethod
    def forward(ctx, img, M, disp, fill=-1000.0, photo=None):
        Mh = _m_host(M)
        out, _ = ops.warp_displacement(img, Mh, disp.contiguous(), fill=fill, photo=photo)
        ctx.save_for_backward(img, disp)
        ctx.Mh, ctx.fill, ctx.M_meta, ctx.photo = Mh, fill, (M.device, M.dtype), photo
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, disp = ctx.saved_tensors
        g_img, g_M, g_disp = ops.warp_displacement_backward(
            img, ctx.Mh, disp.contiguous(), grad_out.contiguous(), fill=ctx.fill,
            want_img=ctx.needs_input_grad[0], want_M=ctx.needs_input_grad[1],
            want_disp=ctx.needs_input_grad[2], photo=ctx.photo)
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, g_disp, None, None


class WarpBsplineFn(torch.autograd.Function):
    """out = warp(img; M, B ctrl) with the B-spline displacement evaluated in
    the warp kernel (photometrics as WarpAffineFn); gradients to img, M and
    the control grid ctrl."""

    @staticmethod
    def forward(ctx, img, M, ctrl, fill=-1000.0, out_dim=None, photo=None):
        Mh = _m_host(M)
        out, _ = ops.warp_bspline(img, Mh, ctrl.contiguous(), fill=fill, out_dim=out_dim,
                                  photo=photo)
        ctx.save_for_backward(img, ctrl)
        ctx.Mh, ctx.fill, ctx.M_meta, ctx.photo = Mh, fill, (M.device, M.dtype), photo
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, ctrl = ctx.saved_tensors
        g_img, g_M, g_ctrl = ops.warp_bspline_backward(
            img, ctx.Mh, ctrl.contiguous(), grad_out.contiguous(), fill=ctx.fill,
            want_img=ctx.needs_input_grad[0], want_M=ctx.needs_input_grad[1],
            want_ctrl=ctx.needs_input_grad[2], photo=ctx.photo)
        if g_M is not None:
            g_M = g_M.to(ctx.M_meta[0], ctx.M_meta[1])
        return g_img, g_M, g_ctrl, None, None, None


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


def warp_displacement(img, M, disp, fill=-1000.0, photo=None):
    return WarpDisplacementFn.apply(img, M, disp, fill, photo)


def warp_bspline(img, M, ctrl, fill=-1000.0, out_dim=None, photo=None):
    return WarpBsplineFn.apply(img, M, ctrl, fill, out_dim, photo)


def bspline_upsample(ctrl, out_dim):
    return BSplineUpsampleFn.apply(ctrl, out_dim)
