"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times, compared whole: every output voxel of
every volume against the oracle on the same inputs.  Same bars as the
small-size parity tests: labels bit-exact, intensities within 1e-5 (scaled),
gradients within 1e-4.  The nonrigid workload is compared against the
oracle on both its FP32 evaluation of the B-spline field and on the plain
FP64 field (tests/field_bounds.py gives the allowances the FP32 field's
rounding bound implies).
"""
import ctypes
import functools

import numpy as np
import pytest
import torch

import bench
import field_bounds as fb
import oracle
import paper_1811_11226_amd as ctaug
from synth import configs

from test_gpu_parity import DEV, _np, _t, assert_grad, assert_intensity

pytestmark = pytest.mark.gpu


def _check_whole(out, lout, img, lbl, M, out_dim, fill, label_fill, photo, what, disp=None):
    ref, lref = oracle.warp(img, M, out_dim, lbl=lbl, disp=disp, fill=fill,
                            label_fill=label_fill, photo=photo)
    windowed = photo is not None and photo.window
    assert_intensity(_np(out), ref, windowed, what)
    if lout is not None:
        assert np.array_equal(_np(lout), lref), f"{what}: labels"


def test_c3_batch_full_size_in_benchmark_launch_shape():
    """The 16-volume batch (int16 inputs U{96..256}^3 -> 120x120x160, labels,
    full photometrics) through the benchmark's own batch plan and launch
    shape: a direct launch on one parameter draw, then a descriptor update
    and HIP-graph replays on another, every volume compared whole."""
    s = bench.C3Set(0, 2, DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s.plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(s.jobs):
        M, ph = s.pool[0][k]
        _check_whole(s.outs[k], s.louts[k], j.img, j.lbl, M, bench.C3_OUT, j.fill,
                     j.label_fill, ph, f"draw 0 volume {k}")
    with torch.cuda.stream(stream):
        s.plan.update(s.job_arrays[1])
        s.plan.capture()
        s.plan.replay()
        s.plan.replay()
    torch.cuda.synchronize()
    for k, j in enumerate(s.jobs):
        M, ph = s.pool[1][k]
        _check_whole(s.outs[k], s.louts[k], j.img, j.lbl, M, bench.C3_OUT, j.fill,
                     j.label_fill, ph, f"draw 1 volume {k}")
    s.plan.close()


def test_c2_full_resolution_volume_whole():
    """512x512x320 int16 volume with labels and full photometrics."""
    j = configs.c2()[0]
    _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
    out, lout = ctaug.warp_affine(_t(j.img), M, lbl=_t(j.lbl), fill=j.fill,
                                  label_fill=j.label_fill, photo=j.photo, out_dim=j.out_dim)
    _check_whole(out, lout, j.img, j.lbl, M, j.out_dim, j.fill, j.label_fill, j.photo,
                 "512x512x320")


def test_c4_batch_forward_and_adjoint_full_size():
    """8 x 128^3 float32: the batched forward (as the benchmark launches it)
    compared whole, and the adjoint to the image and the 12 parameters of
    every volume compared whole."""
    jobs, grads = configs.c4()
    imgs = [_t(j.img) for j in jobs]
    Ms = [ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)[1] for j in jobs]
    outs = [torch.empty(j.out_dim, dtype=torch.float32, device=DEV) for j in jobs]
    plan = ctaug.BatchPlan([ctaug.make_job(imgs[k], Ms[k], outs[k], fill=jobs[k].fill)
                            for k in range(len(jobs))])
    plan.launch()
    for k, j in enumerate(jobs):
        _check_whole(outs[k], None, j.img, None, Ms[k], j.out_dim, j.fill, 0, None,
                     f"c4 forward volume {k}")
    plan.close()
    for k, j in enumerate(jobs):
        g_img, g_M = ctaug.warp_affine_backward(imgs[k], Ms[k], _t(grads[k]), fill=j.fill)
        r_img, r_M, _ = oracle.warp_backward(j.img, Ms[k], grads[k], fill=j.fill)
        assert_grad(_np(g_img), r_img, f"c4 g_img volume {k}")
        assert_grad(_np(g_M), r_M, f"c4 g_M volume {k}")


@functools.lru_cache(maxsize=1)
def _c5():
    return configs.c5()


@pytest.mark.parametrize("k", range(4))
def test_c5_nonrigid_full_size(k):
    """4 x 256^3 float32 with the cubic B-spline field of an 8^3 control grid
    evaluated inside the warp (noise on, as the benchmark runs it), volume k
    compared whole: the forward against the oracle on the FP32 evaluation of
    the field (1e-5) and on the plain FP64 field (1e-5 plus the field
    bound's effect); the fused adjoint (image, parameters, control grid)
    against the oracle's adjoint on the FP32 field, and against the FP64
    field with the upstream gradient zeroed where q lies within the field
    bound of a cell plane (normwise for the image; elementwise for M and the
    control grid with the allowance for dV/dq moving inside its cell)."""
    jobs, ctrls, grads = _c5()
    j, C, g = jobs[k], ctrls[k], grads[k]
    _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
    img = _t(j.img)
    out, _ = ctaug.warp_bspline(img, M, _t(C), fill=j.fill, photo=j.photo)
    got = _np(out)
    u32 = oracle.bspline_upsample_f32(C, j.out_dim)
    ref, _ = oracle.warp(j.img, M, j.out_dim, disp=u32, fill=j.fill, photo=j.photo)
    assert_intensity(got, ref, False, f"c5 forward volume {k} (FP32 field)")
    u_ref = oracle.bspline_upsample(C.astype(np.float64), j.out_dim).astype(np.float32)
    q, d = fb.coords(M, j.out_dim, u_ref), fb.delta(M, j.out_dim, C, u_ref)
    ref64, _ = oracle.warp(j.img, M, j.out_dim, disp=u_ref, fill=j.fill, photo=j.photo)
    fb.assert_values_within_field_slack(got, ref64, j.img, q, d, j.fill, 1000.0,
                                        what=f"c5 forward volume {k} (FP64 field)",
                                        gain=j.photo.gain)
    del got, ref, ref64
    # the fused route
    od = (ctypes.c_int64 * 3)(*j.out_dim)
    G = (ctypes.c_int64 * 3)(*C.shape[1:])
    L = ctaug._lib.load()
    m_bytes = ctaug.ops.warp_backward_workspace(j.out_dim)     # rows x 12 doubles
    rows = m_bytes // 96
    ws_fused = -(-m_bytes // 256) * 256 + (rows + min(rows, 64)) * 3 * int(np.prod(C.shape[1:])) * 8
    assert int(L.ctaug_warp_bspline_backward_workspace(od, G)) == ws_fused
    g_img, g_M, g_c = ctaug.warp_bspline_backward(img, M, _t(C), _t(g), fill=j.fill)
    r_img, r_M, r_u = oracle.warp_backward(j.img, M, g, disp=u32, fill=j.fill, want_u=True)
    assert_grad(_np(g_img), r_img, f"c5 g_img volume {k}")
    assert_grad(_np(g_M), r_M, f"c5 g_M volume {k}")
    assert_grad(_np(g_c), oracle.bspline_adjoint(r_u, C.shape[1:]), f"c5 g_ctrl volume {k}")
    del r_img, r_u
    gm = np.where(fb.near_planes(q, d), np.float32(0), g)
    g_img, g_M, g_c = ctaug.warp_bspline_backward(img, M, _t(C), _t(gm), fill=j.fill)
    r_img, r_M, r_u = oracle.warp_backward(j.img, M, gm, disp=u_ref, fill=j.fill, want_u=True)
    nref = np.linalg.norm(r_img)
    assert np.linalg.norm(_np(g_img) - r_img) <= 1e-4 * nref, f"c5 g_img volume {k} (FP64 field)"
    a = fb.dvdq_slack(j.img, q, d, j.fill, gm)
    fb.assert_grad_masked(_np(g_M), r_M, f"c5 g_M volume {k} (FP64 field)",
                          slack=fb.grad_M_slack(a))
    fb.assert_grad_masked(_np(g_c), oracle.bspline_adjoint(r_u, C.shape[1:]),
                          f"c5 g_ctrl volume {k} (FP64 field)",
                          slack=oracle.bspline_adjoint(np.stack([a] * 3), C.shape[1:]))
