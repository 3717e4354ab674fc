"""The nonrigid comparison helpers (tests/field_bounds.py) on the CPU: the
oracle's own FP32 evaluation of the B-spline field passes them against the
FP64 definition, and planted mistakes in the field or the warp fail them."""
import numpy as np
import pytest

import field_bounds as fb
import oracle
from synth import AugmentRanges, draw_affine_params, phantom_pair


def _case(seed=61, in_dim=(40, 36, 30), out_dim=(37, 29, 23), grid=(6, 7, 5), amp=3.0):
    rng = np.random.default_rng(seed)
    img, lbl = phantom_pair(in_dim, seed=8)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    M = oracle.affine_matrix(prm, in_dim, out_dim).astype(np.float32)
    C = (amp * rng.standard_normal((3,) + grid)).astype(np.float32)
    u_ref = oracle.bspline_upsample(C.astype(np.float64), out_dim).astype(np.float32)
    return rng, img, lbl, M, C, u_ref, out_dim, grid


def test_fp32_field_passes_against_fp64_definition():
    rng, img, lbl, M, C, u_ref, od, grid = _case()
    u32 = oracle.bspline_upsample_f32(C, od)
    q, d = fb.coords(M, od, u_ref), fb.delta(M, od, C, u_ref)
    a, la = oracle.warp(img, M, od, lbl=lbl, disp=u32)
    b, lb = oracle.warp(img, M, od, lbl=lbl, disp=u_ref)
    fb.assert_labels_up_to_ties(la, lb, q, d, lbl, 0)
    fb.assert_values_within_field_slack(a, b, img, q, d, -1000.0, 1000.0)
    g = rng.standard_normal(od).astype(np.float32)
    gm = np.where(fb.near_planes(q, d), np.float32(0), g)
    r = oracle.warp_backward(img, M, gm, disp=u32, want_u=True)
    s = oracle.warp_backward(img, M, gm, disp=u_ref, want_u=True)
    fb.assert_grad_masked(r[1], s[1], "g_M")
    fb.assert_grad_masked(oracle.bspline_adjoint(r[2], grid), oracle.bspline_adjoint(s[2], grid))
    ri = oracle.warp_backward(img, M, g, disp=u32, want_M=False)[0]
    si = oracle.warp_backward(img, M, g, disp=u_ref, want_M=False)[0]
    slack = 3.0 * d.max() * fb.corner_abs_sums(q, np.abs(g.astype(np.float64)), img.shape)
    fb.assert_grad_masked(ri, si, "g_img", slack=slack)


@pytest.mark.parametrize("mistake", ["shift", "transposed_grid", "sign"])
def test_planted_field_mistakes_fail(mistake):
    rng, img, lbl, M, C, u_ref, od, grid = _case(seed=62)
    if mistake == "shift":             # a field off by a hundredth of a voxel
        u_bad = u_ref + np.float32(0.01)
    elif mistake == "transposed_grid":  # control grid read with x and z swapped
        Ct = np.ascontiguousarray(np.transpose(C, (0, 3, 2, 1)))
        u_bad = oracle.bspline_upsample(Ct.astype(np.float64), od).astype(np.float32)
    else:                              # the displacement subtracted
        u_bad = -u_ref
    q, d = fb.coords(M, od, u_ref), fb.delta(M, od, C, u_ref)
    a, la = oracle.warp(img, M, od, lbl=lbl, disp=u_bad)
    b, lb = oracle.warp(img, M, od, lbl=lbl, disp=u_ref)
    with pytest.raises(AssertionError):
        fb.assert_values_within_field_slack(a, b, img, q, d, -1000.0, 1000.0)
    with pytest.raises(AssertionError):
        fb.assert_labels_up_to_ties(la, lb, q, d, lbl, 0)


def test_corner_spread_equals_brute_force():
    rng = np.random.default_rng(5)
    img = rng.integers(-1000, 1000, (7, 6, 5)).astype(np.float64)
    q = rng.uniform(-2.5, 8.5, (3, 40))
    d = np.array([1e-3, 2e-3, 5e-4])
    got = fb.corner_spread(img, q, d, -1000.0)
    for m in range(q.shape[1]):
        vals = []
        for a in range(3):
            for b in range(3):
                for c in range(3):
                    j = [int(np.floor(q[i, m] - d[i])) + o for i, o in enumerate((a, b, c))]
                    inside = all(0 <= j[i] < img.shape[i] for i in range(3))
                    vals.append(img[tuple(j)] if inside else -1000.0)
        assert got[m] == max(vals) - min(vals)
