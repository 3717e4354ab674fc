"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times.

Where the oracle cannot finish a whole workload in seconds (the 16-volume
batch with photometrics, the 512x512x320 volume, the 256^3 nonrigid warp) it
evaluates sampled output voxels one by one: first and last voxels, whole z
rows across tile borders, and uniformly drawn voxels.  The 8 x 128^3 forward
and its adjoint are compared whole.  Same bars as the small-size parity
tests: labels bit-exact, intensities within 1e-5 (scaled), gradients within
1e-4.
"""
import ctypes

import numpy as np
import pytest
import torch

import bench
import oracle
import paper_1811_11226_amd as ctaug
from synth import configs

from test_gpu_parity import DEV, _np, _t, assert_grad, assert_intensity

pytestmark = pytest.mark.gpu


def _sample(out_dim, rng, n_random=3000, n_rows=6):
    """Linear output indices: first and last voxel, n_rows whole z rows (the
    first and last rows included) and n_random uniform draws."""
    X, Y, Z = out_dim
    n = X * Y * Z
    rows = [(0, 0), (X - 1, Y - 1)] + [tuple(rng.integers(0, (X, Y))) for _ in range(n_rows - 2)]
    parts = [np.array([0, n - 1], np.int64), rng.integers(0, n, size=n_random)]
    for x, y in rows:
        parts.append((int(x) * Y + int(y)) * Z + np.arange(Z, dtype=np.int64))
    return np.concatenate(parts)


def _check_points(out, lout, job_img, job_lbl, M, out_dim, fill, label_fill, photo, idx,
                  disp=None, what=""):
    ref, lref = oracle.warp_points(job_img, M, out_dim, idx, lbl=job_lbl, disp=disp, fill=fill,
                                   label_fill=label_fill, photo=photo)
    got = _np(out).ravel()[idx]
    windowed = photo is not None and photo.window
    assert_intensity(got, ref, windowed, what)
    if lout is not None:
        assert np.array_equal(_np(lout).ravel()[idx], lref), f"{what}: labels"


def test_c3_batch_full_size_in_benchmark_launch_shape():
    """The 16-volume batch (int16 inputs U{96..256}^3 -> 120x120x160, labels,
    full photometrics) through the benchmark's own batch plan and launch
    shape: a direct launch on one parameter draw, then a descriptor update
    and HIP-graph replays on another, each checked on sampled voxels of
    every volume."""
    s = bench.C3Set(0, 2, DEV)
    rng = np.random.default_rng(303)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s.plan.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(s.jobs):
        M, ph = s.pool[0][k]
        idx = _sample(bench.C3_OUT, rng, n_random=1500, n_rows=4)
        _check_points(s.outs[k], s.louts[k], j.img, j.lbl, M, bench.C3_OUT, j.fill,
                      j.label_fill, ph, idx, what=f"draw 0 volume {k}")
    with torch.cuda.stream(stream):
        s.plan.update(s.job_arrays[1])
        s.plan.capture()
        s.plan.replay()
        s.plan.replay()
    torch.cuda.synchronize()
    for k, j in enumerate(s.jobs):
        M, ph = s.pool[1][k]
        idx = _sample(bench.C3_OUT, rng, n_random=1500, n_rows=4)
        _check_points(s.outs[k], s.louts[k], j.img, j.lbl, M, bench.C3_OUT, j.fill,
                      j.label_fill, ph, idx, what=f"draw 1 volume {k}")
    s.plan.close()


def test_c2_full_resolution_volume_sampled():
    """512x512x320 int16 volume with labels and full photometrics."""
    j = configs.c2()[0]
    _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
    out, lout = ctaug.warp_affine(_t(j.img), M, lbl=_t(j.lbl), fill=j.fill,
                                  label_fill=j.label_fill, photo=j.photo, out_dim=j.out_dim)
    idx = _sample(j.out_dim, np.random.default_rng(202), n_random=20000, n_rows=8)
    _check_points(out, lout, j.img, j.lbl, M, j.out_dim, j.fill, j.label_fill, j.photo, idx,
                  what="512x512x320")


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
        ref, _ = oracle.warp(j.img, Ms[k], j.out_dim, fill=j.fill)
        assert_intensity(_np(outs[k]), ref, False, f"c4 forward volume {k}")
    plan.close()
    for k, j in enumerate(jobs):
        g_img, g_M = ctaug.warp_affine_backward(imgs[k], Ms[k], _t(grads[k]), fill=j.fill)
        r_img, r_M, _ = oracle.warp_backward(j.img, Ms[k], grads[k], fill=j.fill)
        assert_grad(_np(g_img), r_img, f"c4 g_img volume {k}")
        assert_grad(_np(g_M), r_M, f"c4 g_M volume {k}")


def test_c5_nonrigid_full_size():
    """4 x 256^3 float32 with the cubic B-spline field of an 8^3 control grid
    evaluated inside the warp: the forward of every volume on sampled voxels
    against the oracle on its FP32 parity-mode field, and the fused adjoint
    (image, parameters, control grid) of the first volume compared whole."""
    jobs, ctrls, grads = configs.c5()
    rng = np.random.default_rng(505)
    for k, j in enumerate(jobs):
        _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
        out = ctaug.warp_bspline(_t(j.img), M, _t(ctrls[k]), fill=j.fill, photo=j.photo)
        out = out[0] if isinstance(out, tuple) else out
        u = oracle.bspline_upsample_f32(ctrls[k], j.out_dim)
        idx = _sample(j.out_dim, rng, n_random=5000, n_rows=6)
        _check_points(out, None, j.img, None, M, j.out_dim, j.fill, 0, j.photo, idx, disp=u,
                      what=f"c5 forward volume {k}")
    j, C, g = jobs[0], ctrls[0], grads[0]
    _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
    od = (ctypes.c_int64 * 3)(*j.out_dim)
    G = (ctypes.c_int64 * 3)(*C.shape[1:])
    L = ctaug._lib.load()
    m_bytes = ctaug.ops.warp_backward_workspace(j.out_dim)     # rows x 12 doubles
    rows = m_bytes // 96
    ws_fused = -(-m_bytes // 256) * 256 + (rows + min(rows, 64)) * 3 * int(np.prod(C.shape[1:])) * 8
    assert int(L.ctaug_warp_bspline_backward_workspace(od, G)) == ws_fused   # the fused route
    g_img, g_M, g_c = ctaug.warp_bspline_backward(_t(j.img), M, _t(C), _t(g), fill=j.fill)
    u = oracle.bspline_upsample_f32(C, j.out_dim)
    r_img, r_M, r_u = oracle.warp_backward(j.img, M, g, disp=u, fill=j.fill, want_u=True)
    assert_grad(_np(g_img), r_img, "c5 g_img")
    assert_grad(_np(g_M), r_M, "c5 g_M")
    assert_grad(_np(g_c), oracle.bspline_adjoint(r_u, C.shape[1:]), "c5 g_ctrl")
