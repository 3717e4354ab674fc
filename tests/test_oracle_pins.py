"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the property it checks: closed forms (identity, integer
shifts, axis permutations, linear ramps, scale 2 / scale 1/2, the centre
formula), invariants (constants, adjoint identity, mass conservation,
partition of unity), brute force on tiny inputs (dense tent-weight matrix,
nearest-voxel search), independent library routines (SciPy ndimage, torch CPU
grid_sample and autograd, SciPy rotations, rocRAND's host Philox engine),
finite differences of the gradients, statistics of the noise, and the window
examples printed in the paper (tests/golden/window_examples.txt).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.stats
from scipy.spatial.transform import Rotation

import oracle
from synth import AugmentRanges, PhotoParams, draw_affine_params, identity_affine_params, phantom_pair

HERE = os.path.dirname(os.path.abspath(__file__))
FILL = -1000.0


def _rand_img(rng, dims, lo=-1000, hi=1500):
    return rng.integers(lo, hi + 1, size=dims).astype(np.float64)


def _M(A, b):
    M = np.zeros((3, 4))
    M[:, :3] = A
    M[:, 3] = b
    return M.ravel()


def _dyadic_M(rng, in_dim=(8, 8, 8), out_dim=None, scale_range=(0.7, 1.4), shift=3.0, denom=64):
    """A random rotation*scale about the volume centres plus a shift, rounded to
    multiples of 1/denom so that the FP32 fma chain of the coordinate map is
    exact for small volumes."""
    out_dim = in_dim if out_dim is None else out_dim
    R = Rotation.random(random_state=int(rng.integers(1 << 31))).as_matrix()
    A = R * rng.uniform(*scale_range)
    c_in = (np.array(in_dim) - 1) / 2
    c_out = (np.array(out_dim) - 1) / 2
    b = c_in - A @ c_out + rng.uniform(-shift, shift, 3)
    return np.round(_M(A, b) * denom) / denom


def _coords_exact(M, out_dim):
    M = np.asarray(M, dtype=np.float64).reshape(3, 4)
    g = np.indices(out_dim).reshape(3, -1).astype(np.float64)
    return (M[:, :3] @ g + M[:, 3:4])  # 3 x N


# --------------------------------------------------------------------------
# C-P1 .. C-P3: identity, integer translation, exact axis permutations/flips
# --------------------------------------------------------------------------

def test_identity_is_bit_exact():
    img, lbl = phantom_pair((13, 11, 9), seed=5)
    M = _M(np.eye(3), np.zeros(3))
    out, lout = oracle.warp(img, M, img.shape, lbl=lbl, fill=123.0)
    assert np.array_equal(out, img.astype(np.float64))
    assert np.array_equal(lout, lbl)


@pytest.mark.parametrize("shift", [(1, 0, 0), (0, -2, 0), (0, 0, 3), (2, -1, -3), (20, 0, 0)])
def test_integer_translation_is_exact_shift(shift):
    img, lbl = phantom_pair((10, 9, 8), seed=7)
    M = _M(np.eye(3), np.array(shift, dtype=np.float64))
    out, lout = oracle.warp(img, M, img.shape, lbl=lbl, fill=FILL, label_fill=0)
    ref = np.full(img.shape, FILL)
    lref = np.zeros(img.shape, dtype=np.int8)
    X, Y, Z = img.shape
    for x in range(X):
        for y in range(Y):
            for z in range(Z):
                s = (x + shift[0], y + shift[1], z + shift[2])
                if all(0 <= s[i] < img.shape[i] for i in range(3)):
                    ref[x, y, z] = img[s]
                    lref[x, y, z] = lbl[s]
    assert np.array_equal(out, ref)
    assert np.array_equal(lout, lref)


def _perm_cases():
    # (A, numpy reference transform) for out(p) = in(A p + b), b = c - A c
    return [
        ("rot90_z", np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]), lambda a: np.rot90(a, k=-1, axes=(0, 1))),
        ("rot90_x", np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]]), lambda a: np.rot90(a, k=-1, axes=(1, 2))),
        ("flip_x", np.diag([-1, 1, 1]), lambda a: a[::-1]),
        ("flip_yz", np.diag([1, -1, -1]), lambda a: a[:, ::-1, ::-1]),
        ("swap_xz", np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]]), lambda a: np.transpose(a, (2, 1, 0))),
    ]


@pytest.mark.parametrize("name,A,ref", _perm_cases(), ids=[c[0] for c in _perm_cases()])
def test_exact_axis_permutations(name, A, ref):
    n = 8
    img, lbl = phantom_pair((n, n, n), seed=11)
    c = np.full(3, (n - 1) / 2)
    b = c - A @ c
    assert np.all(b == np.round(b))
    M = _M(A.astype(np.float64), b)
    out, lout = oracle.warp(img, M, img.shape, lbl=lbl)
    # out[p] = in[A p + b]: build the expectation by explicit indexing
    exp = np.empty_like(img, dtype=np.float64)
    lexp = np.empty_like(lbl)
    for p in np.ndindex(img.shape):
        s = tuple((A @ np.array(p) + b).astype(int))
        exp[p] = img[s]
        lexp[p] = lbl[s]
    assert np.array_equal(out, exp)
    assert np.array_equal(lout, lexp)
    # and the explicit expectation equals the named NumPy operation
    assert np.array_equal(exp, ref(img).astype(np.float64))


# --------------------------------------------------------------------------
# C-P4 .. C-P6: constants, linear ramps, scale 2 and scale 1/2
# --------------------------------------------------------------------------

def test_constant_volume_preserved():
    rng = np.random.default_rng(3)
    dims = (9, 10, 11)
    C = 437.0
    img = np.full(dims, C)
    M = _dyadic_M(rng, dims, shift=2.0)
    out, _ = oracle.warp(img, M, dims, fill=FILL)
    q = _coords_exact(M, dims).T.reshape(dims + (3,))
    inside = np.all((q >= 0) & (q <= np.array(dims) - 1), axis=-1)
    assert inside.sum() > 50
    assert np.all(out[inside] == C)
    # with C == fill, the value is C everywhere, inside or not
    out2, _ = oracle.warp(np.full(dims, FILL), M, dims, fill=FILL)
    assert np.all(out2 == FILL)


def test_linear_ramp_reproduced_and_gradient_closed_form():
    rng = np.random.default_rng(4)
    dims = (12, 10, 14)
    al, be, ga, de = 3.25, -1.5, 0.75, 10.0
    X, Y, Z = np.indices(dims).astype(np.float64)
    img = al * X + be * Y + ga * Z + de
    M = _dyadic_M(rng, dims, shift=2.0)
    out, _ = oracle.warp(img, M, dims, fill=FILL)
    q = _coords_exact(M, dims)
    ramp = (al * q[0] + be * q[1] + ga * q[2] + de).reshape(dims)
    inside = np.all((q >= 0) & (q <= (np.array(dims) - 1)[:, None]), axis=0).reshape(dims)
    assert inside.sum() > 100
    np.testing.assert_allclose(out[inside], ramp[inside], rtol=0, atol=1e-10)
    # gradient w.r.t. M on voxels whose whole cell is inside: dV/dq = (al, be, ga)
    strict = np.all((q >= 0) & (q < (np.array(dims) - 1)[:, None]), axis=0).reshape(dims)
    g = np.where(strict, rng.standard_normal(dims), 0.0)
    _, gM, _ = oracle.warp_backward(img, M, g, fill=FILL)
    P = np.concatenate([np.indices(dims).reshape(3, -1), np.ones((1, g.size))]).astype(np.float64)
    coef = np.array([al, be, ga])
    ref = (coef[:, None] * (P @ g.ravel())[None, :]).ravel()
    np.testing.assert_allclose(gM, ref, rtol=1e-12, atol=1e-9)


def test_scale_two_subsamples_exactly():
    img, lbl = phantom_pair((16, 14, 12), seed=13)
    M = _M(2 * np.eye(3), np.zeros(3))
    out, lout = oracle.warp(img, M, (8, 7, 6), lbl=lbl)
    assert np.array_equal(out, img[::2, ::2, ::2].astype(np.float64))
    assert np.array_equal(lout, lbl[::2, ::2, ::2])


def test_scale_half_midpoints_and_ties_round_up():
    img, lbl = phantom_pair((6, 5, 4), seed=17)
    img = img.astype(np.float64)
    M = _M(0.5 * np.eye(3), np.zeros(3))
    od = (11, 9, 7)
    out, lout = oracle.warp(img, M, od, lbl=lbl)
    # exact midpoint averages: the trilinear value at half-integer points is the
    # mean of the (2 or 4 or 8) neighbouring voxels
    for p in np.ndindex(od):
        lo = [pi // 2 for pi in p]
        hi = [(pi + 1) // 2 for pi in p]
        block = img[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        assert out[p] == pytest.approx(block.mean(), abs=1e-12)
        # q = p/2: ties at .5 resolve upward
        assert lout[p] == lbl[tuple(hi)]


# --------------------------------------------------------------------------
# C-P7, C-P8: brute-force dense W (tent-weight form), adjoint identity, mass
# --------------------------------------------------------------------------

def _dense_W(M, in_dim, out_dim):
    """W[p, c] = prod_i max(0, 1 - |q_i(p) - c_i|) over in-volume voxels c: the
    tent-function form of trilinear weights, independent of floor/lerp."""
    q = _coords_exact(M, out_dim)  # exact for dyadic M
    cs = np.indices(in_dim).reshape(3, -1).astype(np.float64)
    W = np.ones((q.shape[1], cs.shape[1]))
    for i in range(3):
        W *= np.maximum(0.0, 1.0 - np.abs(q[i][:, None] - cs[i][None, :]))
    return W, q


def _nearest_brute(q, in_dim, lbl, label_fill=0):
    out = np.empty(q.shape[1], dtype=np.int8)
    for k in range(q.shape[1]):
        j = []
        for i in range(3):
            cand = np.arange(-3, in_dim[i] + 3)
            d = np.abs(q[i, k] - cand)
            best = cand[d == d.min()].max()   # nearest, ties to the larger index
            j.append(best)
        ok = all(0 <= j[i] < in_dim[i] for i in range(3))
        out[k] = lbl[tuple(j)] if ok else label_fill
    return out


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_dense_W(seed):
    rng = np.random.default_rng(100 + seed)
    in_dim = tuple(int(v) for v in rng.integers(4, 9, 3))
    out_dim = tuple(int(v) for v in rng.integers(4, 9, 3))
    M = _dyadic_M(rng, in_dim, out_dim, shift=2.5)
    img = _rand_img(rng, in_dim)
    lbl = rng.integers(0, 6, in_dim).astype(np.int8)
    fill = float(rng.uniform(-1000, 1000))
    W, q = _dense_W(M, in_dim, out_dim)
    out, lout = oracle.warp(img, M, out_dim, lbl=lbl, fill=fill)
    ref = W @ img.ravel() + fill * (1.0 - W.sum(axis=1))
    np.testing.assert_allclose(out.ravel(), ref, rtol=1e-13, atol=1e-9)
    assert np.array_equal(lout.ravel(), _nearest_brute(q, in_dim, lbl))
    y = rng.standard_normal(out_dim)
    g_img, _, _ = oracle.warp_backward(img, M, y, fill=fill)
    np.testing.assert_allclose(g_img.ravel(), W.T @ y.ravel(), rtol=1e-12, atol=1e-12)


def test_adjoint_identity_and_mass_conservation():
    rng = np.random.default_rng(8)
    in_dim, out_dim = (17, 15, 13), (14, 16, 12)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    M = oracle.affine_matrix(prm, in_dim, out_dim)
    x = rng.standard_normal(in_dim)
    y = rng.standard_normal(out_dim)
    Wx, _ = oracle.warp(x, M, out_dim, fill=0.0)
    WTy, _, _ = oracle.warp_backward(x, M, y, fill=0.0, want_M=False)
    lhs, rhs = np.vdot(Wx, y), np.vdot(x, WTy)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(Wx).ravel() @ np.abs(y).ravel())
    # mass: sum_c (W^T y)_c = sum_p y_p * (sum of in-volume weights of p) = <W 1, y>
    W1, _ = oracle.warp(np.ones(in_dim), M, out_dim, fill=0.0)
    assert WTy.sum() == pytest.approx(np.vdot(W1, y), rel=1e-12, abs=1e-12)


# --------------------------------------------------------------------------
# C-P9, C-P10: SciPy ndimage and torch CPU grid_sample cross-checks
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_scipy_affine_transform_dyadic(seed):
    rng = np.random.default_rng(200 + seed)
    in_dim, out_dim = (14, 12, 10), (12, 13, 11)
    img, lbl = phantom_pair(in_dim, seed=300 + seed)
    img = img.astype(np.float64)
    M = _dyadic_M(rng, in_dim, out_dim, shift=3.0)
    A, b = M.reshape(3, 4)[:, :3], M.reshape(3, 4)[:, 3]
    out, _ = oracle.warp(img, M, out_dim, fill=FILL)
    ref = ndi.affine_transform(img, A, offset=b, output_shape=out_dim, order=1,
                               mode="grid-constant", cval=FILL)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-9)


def test_scipy_affine_transform_general_and_labels():
    rng = np.random.default_rng(9)
    in_dim, out_dim = (20, 18, 16), (18, 18, 18)
    img, lbl = phantom_pair(in_dim, seed=21)
    img = img.astype(np.float64)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    M32 = oracle.affine_matrix(prm, in_dim, out_dim).astype(np.float32)
    A, b = M32.astype(np.float64).reshape(3, 4)[:, :3], M32.astype(np.float64).reshape(3, 4)[:, 3]
    out, lout = oracle.warp(img, M32, out_dim, lbl=lbl, fill=FILL)
    ref = ndi.affine_transform(img, A, offset=b, output_shape=out_dim, order=1,
                               mode="grid-constant", cval=FILL)
    # SciPy maps coordinates in FP64, the oracle in pinned FP32: the values
    # differ by at most |grad I| * |dq| with |dq| <~ 2^-24 * |q| * 4
    q = _coords_exact(M32, out_dim)
    dq = 4 * 2.0 ** -24 * (np.abs(q).max() + 1)
    assert np.max(np.abs(out - ref)) <= 2500.0 * dq * 3
    lref = ndi.affine_transform(lbl, A, offset=b, output_shape=out_dim, order=0,
                                mode="grid-constant", cval=0)
    frac = np.abs(q - np.round(q)).reshape(3, *out_dim)
    near_tie = np.any(np.abs(frac - 0.5) < 1e-4, axis=0)
    assert np.array_equal(lout[~near_tie], lref[~near_tie])


def _torch_warp(img, M, out_dim, fill, g=None):
    import torch
    t_img = torch.tensor(img, dtype=torch.float64, requires_grad=True)
    t_M = torch.tensor(np.asarray(M, dtype=np.float64).reshape(3, 4), requires_grad=True)
    P = torch.tensor(np.concatenate([np.indices(out_dim).reshape(3, -1),
                                     np.ones((1, int(np.prod(out_dim))))]), dtype=torch.float64)
    q = t_M @ P                                    # 3 x N
    n = torch.tensor(img.shape, dtype=torch.float64)[:, None]
    gn = 2.0 * q / (n - 1.0) - 1.0                 # align_corners=True normalisation
    grid = torch.stack([gn[2], gn[1], gn[0]], dim=-1).reshape(1, *out_dim, 3)
    v = torch.nn.functional.grid_sample((t_img - fill)[None, None], grid, mode="bilinear",
                                        padding_mode="zeros", align_corners=True)[0, 0] + fill
    if g is None:
        return v.detach().numpy(), None, None
    (v * torch.tensor(g, dtype=torch.float64)).sum().backward()
    return v.detach().numpy(), t_img.grad.numpy(), t_M.grad.numpy().ravel()


@pytest.mark.parametrize("seed", range(3))
def test_torch_grid_sample_forward_and_backward(seed):
    rng = np.random.default_rng(400 + seed)
    in_dim, out_dim = (15, 13, 11), (12, 14, 10)
    img = _rand_img(rng, in_dim)
    prm = draw_affine_params(rng, AugmentRanges(disp=(2.0, 2.0, 2.0)), in_dim, out_dim)
    M = oracle.affine_matrix(prm, in_dim, out_dim)
    g = rng.standard_normal(out_dim)
    v_ref, gimg_ref, gM_ref = _torch_warp(img, M, out_dim, FILL, g)
    out, _ = oracle.warp(img, M, out_dim, fill=FILL, exact=True)
    np.testing.assert_allclose(out, v_ref, rtol=0, atol=1e-9)
    g_img, g_M, _ = oracle.warp_backward(img, M, g, fill=FILL, exact=True)
    np.testing.assert_allclose(g_img, gimg_ref, rtol=0, atol=1e-10)
    np.testing.assert_allclose(g_M, gM_ref, rtol=1e-9, atol=1e-7 * np.abs(gM_ref).max())


# --------------------------------------------------------------------------
# Gradients: FP64 finite differences in exact mode (C-A17 protocol)
# --------------------------------------------------------------------------

def test_param_gradient_finite_differences():
    rng = np.random.default_rng(12)
    dims = (16, 16, 16)
    img = _rand_img(rng, dims)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims)
    _, g_M, _ = oracle.warp_backward(img, M, g, fill=FILL, exact=True)
    h = 1e-6
    fd = np.zeros(12)
    for k in range(12):
        Mp, Mm = M.copy(), M.copy()
        Mp[k] += h
        Mm[k] -= h
        # reject the instance if any voxel changes cell between the two points
        qp, qm = _coords_exact(Mp, dims), _coords_exact(Mm, dims)
        assert np.array_equal(np.floor(qp), np.floor(qm)), "kink crossed; redraw"
        vp, _ = oracle.warp(img, Mp, dims, fill=FILL, exact=True)
        vm, _ = oracle.warp(img, Mm, dims, fill=FILL, exact=True)
        fd[k] = (np.vdot(vp, g) - np.vdot(vm, g)) / (2 * h)
    np.testing.assert_allclose(g_M, fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max())


def test_image_gradient_finite_differences():
    rng = np.random.default_rng(13)
    dims = (16, 16, 16)
    img = _rand_img(rng, dims)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims)
    g_img, _, _ = oracle.warp_backward(img, M, g, fill=FILL, exact=True, want_M=False)
    for c in [(8, 8, 8), (0, 5, 9), (15, 15, 0), (3, 12, 7)]:
        ip, im = img.copy(), img.copy()
        ip[c] += 1.0
        im[c] -= 1.0
        vp, _ = oracle.warp(ip, M, dims, fill=FILL, exact=True)
        vm, _ = oracle.warp(im, M, dims, fill=FILL, exact=True)
        fd = (np.vdot(vp, g) - np.vdot(vm, g)) / 2.0
        assert g_img[c] == pytest.approx(fd, rel=1e-9, abs=1e-9)


def test_photometric_adjoint_finite_differences():
    """The adjoint with the photometric chain (gain, offset, noise and an
    occluded slab, no window): FD of the noisy, occluded forward in the image
    and in M against the adjoint of gain * g off the slab."""
    rng = np.random.default_rng(16)
    dims = (16, 16, 16)
    img = _rand_img(rng, dims)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    ph = PhotoParams(gain=1.0625, offset=-7.5, sigma=10.0, window=False, seed=44, volume_id=3,
                     occlude=True, occ_lo=4.0, occ_hi=9.5)
    g = rng.standard_normal(dims)
    g_img, g_M, _ = oracle.warp_backward(img, M, g, fill=FILL, exact=True, photo=ph)
    gv = oracle.photometric_adjoint(g, ph)
    z = np.arange(dims[2])
    assert not gv[:, :, (z >= 4) & (z <= 9)].any()
    np.testing.assert_array_equal(gv[:, :, :4], 1.0625 * g[:, :, :4])
    for c in [(8, 8, 8), (3, 12, 7)]:
        ip, im = img.copy(), img.copy()
        ip[c] += 1.0
        im[c] -= 1.0
        vp, _ = oracle.warp(ip, M, dims, fill=FILL, exact=True, photo=ph)
        vm, _ = oracle.warp(im, M, dims, fill=FILL, exact=True, photo=ph)
        fd = (np.vdot(vp, g) - np.vdot(vm, g)) / 2.0
        assert g_img[c] == pytest.approx(fd, rel=1e-9, abs=1e-9)
    h = 1e-6
    for k in (0, 5, 11):
        Mp, Mm = M.copy(), M.copy()
        Mp[k] += h
        Mm[k] -= h
        vp, _ = oracle.warp(img, Mp, dims, fill=FILL, exact=True, photo=ph)
        vm, _ = oracle.warp(img, Mm, dims, fill=FILL, exact=True, photo=ph)
        fd = (np.vdot(vp, g) - np.vdot(vm, g)) / (2 * h)
        assert g_M[k] == pytest.approx(fd, rel=1e-5, abs=1e-5 * np.abs(g_M).max())
    with pytest.raises(Exception):
        oracle.photometric_adjoint(g, PhotoParams(window=True))


def test_displacement_gradient_finite_differences():
    rng = np.random.default_rng(14)
    dims = (12, 12, 12)
    img = _rand_img(rng, dims)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    disp = rng.uniform(-1.5, 1.5, (3,) + dims).astype(np.float32)
    g = rng.standard_normal(dims)
    _, _, g_u = oracle.warp_backward(img, M, g, disp=disp, fill=FILL, exact=True, want_M=False,
                                     want_img=False, want_u=True)
    h = 1e-3
    for comp, p in [(0, (5, 5, 5)), (1, (2, 9, 4)), (2, (10, 3, 7))]:
        dp, dm = disp.copy(), disp.copy()
        dp[(comp,) + p] += h
        dm[(comp,) + p] -= h
        vp, _ = oracle.warp(img, M, dims, disp=dp, fill=FILL, exact=True)
        vm, _ = oracle.warp(img, M, dims, disp=dm, fill=FILL, exact=True)
        fd = (np.vdot(vp, g) - np.vdot(vm, g)) / (2 * h)
        assert g_u[(comp,) + p] == pytest.approx(fd, rel=1e-4, abs=1e-6)


def test_constant_displacement_equals_shift():
    rng = np.random.default_rng(15)
    dims = (10, 11, 12)
    img, lbl = phantom_pair(dims, seed=33)
    M = _dyadic_M(rng, dims, shift=2.0)
    t = np.array([1.25, -2.0, 0.5])
    disp = np.broadcast_to(t[:, None, None, None], (3,) + dims).astype(np.float32).copy()
    Ms = M.reshape(3, 4).copy()
    Ms[:, 3] += t
    a, la = oracle.warp(img, M, dims, lbl=lbl, disp=disp)
    b, lb = oracle.warp(img, Ms.ravel(), dims, lbl=lbl)
    assert np.array_equal(a, b) and np.array_equal(la, lb)


def test_point_sampled_warp_equals_whole_volume_warp():
    """The point-sampled entry (used at sizes where the whole volume is too slow
    for the oracle) indexes output voxels as the whole-volume warp does."""
    rng = np.random.default_rng(16)
    in_dim, out_dim = (14, 12, 10), (9, 13, 11)
    img, lbl = phantom_pair(in_dim, seed=34)
    M = _dyadic_M(rng, in_dim, out_dim)
    disp = rng.normal(0.0, 1.5, size=(3,) + out_dim).astype(np.float32)
    ph = PhotoParams(gain=1.05, offset=7.0, sigma=10.0, window=True, gamma=0.9, seed=11,
                     volume_id=3)
    n = int(np.prod(out_dim))
    idx = np.concatenate([[0, n - 1], rng.integers(0, n, size=200)])
    for d in (None, disp):
        full, lfull = oracle.warp(img, M, out_dim, lbl=lbl, disp=d, photo=ph)
        pts, lpts = oracle.warp_points(img, M, out_dim, idx, lbl=lbl, disp=d, photo=ph)
        assert np.array_equal(pts, full.ravel()[idx]) and np.array_equal(lpts, lfull.ravel()[idx])
    e, le = oracle.warp_points(img, M, out_dim, np.zeros(0, np.int64), lbl=lbl)
    assert e.size == 0 and le.size == 0
    for bad in (-1, n):
        with pytest.raises(ValueError):
            oracle.warp_points(img, M, out_dim, np.array([bad]))


# --------------------------------------------------------------------------
# C-P15 and the transform sampler: centre formula, rotations vs SciPy
# --------------------------------------------------------------------------

def test_centre_displacement_formula():
    rng = np.random.default_rng(16)
    for _ in range(20):
        in_dim = tuple(int(v) for v in rng.integers(96, 257, 3))
        out_dim = (120, 120, 160)
        prm = draw_affine_params(rng, AugmentRanges(shear=(0.1, 0.1, 0.1),
                                                    reflect_prob=(0.5, 0.5, 0.5), generic=0.05),
                                 in_dim, out_dim)
        M = oracle.affine_matrix(prm, in_dim, out_dim).reshape(3, 4)
        c_in = (np.array(in_dim) - 1) / 2
        c_out = (np.array(out_dim) - 1) / 2
        lhs = M[:, :3] @ c_out + M[:, 3]
        np.testing.assert_allclose(lhs, c_in + prm[21:24] + prm[24:27], rtol=0, atol=1e-10)


def test_rotation_composition_matches_scipy():
    rng = np.random.default_rng(17)
    for _ in range(10):
        prm = identity_affine_params()
        prm[0:3] = rng.uniform(-np.pi, np.pi, 3)
        s = rng.uniform(0.8, 1.2)
        prm[3:6] = s
        M = oracle.affine_matrix(prm, (9, 9, 9), (9, 9, 9)).reshape(3, 4)
        # intrinsic z-y'-x'' Euler angles: R = Rz(tz) Ry(ty) Rx(tx)
        R = Rotation.from_euler("ZYX", [prm[2], prm[1], prm[0]]).as_matrix()
        np.testing.assert_allclose(M[:, :3], s * R, rtol=0, atol=1e-14)
        assert np.linalg.det(M[:, :3]) == pytest.approx(s ** 3, rel=1e-12)


def test_reflection_and_shear_structure():
    prm = identity_affine_params()
    prm[9:12] = [1.0, 0.0, 1.0]
    M = oracle.affine_matrix(prm, (8, 8, 8), (8, 8, 8)).reshape(3, 4)
    np.testing.assert_array_equal(M[:, :3], np.diag([-1.0, 1.0, -1.0]))
    np.testing.assert_array_equal(M[:, 3], [7.0, 0.0, 7.0])   # reflection about the centre
    prm = identity_affine_params()
    prm[6:9] = [0.25, -0.5, 0.125]
    M = oracle.affine_matrix(prm, (8, 8, 8), (8, 8, 8)).reshape(3, 4)
    np.testing.assert_array_equal(M[:, :3], [[1, 0.25, -0.5], [0, 1, 0.125], [0, 0, 1]])


# --------------------------------------------------------------------------
# C-P11: cubic B-spline displacement
# --------------------------------------------------------------------------

def test_bspline_matches_scipy_map_coordinates():
    rng = np.random.default_rng(18)
    G = (8, 7, 9)
    out_dim = (17, 13, 10)
    C = rng.standard_normal((3,) + G)
    u = oracle.bspline_upsample(C, out_dim)
    h = [(out_dim[k] - 1) / (G[k] - 3) for k in range(3)]
    pts = np.indices(out_dim).reshape(3, -1).astype(np.float64)
    coords = np.stack([pts[k] / h[k] + 1.0 for k in range(3)])
    for comp in range(3):
        ref = ndi.map_coordinates(C[comp], coords, order=3, prefilter=False, mode="nearest")
        np.testing.assert_allclose(u[comp].ravel(), ref, rtol=0, atol=1e-12)


def test_bspline_partition_of_unity_and_linear_precision():
    G = (8, 8, 8)
    out_dim = (21, 16, 11)
    u = oracle.bspline_upsample(np.full((3,) + G, 2.5), out_dim)
    np.testing.assert_allclose(u, 2.5, rtol=0, atol=1e-13)
    h = [(out_dim[k] - 1) / (G[k] - 3) for k in range(3)]
    J = np.indices(G).astype(np.float64)
    al = (0.3, -1.1, 0.7)
    C = np.stack([sum(al[k] * (J[k] - 1) * h[k] for k in range(3)) + 4.0] * 3)
    u = oracle.bspline_upsample(C, out_dim)
    P = np.indices(out_dim).astype(np.float64)
    ref = sum(al[k] * P[k] for k in range(3)) + 4.0
    for comp in range(3):
        np.testing.assert_allclose(u[comp], ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("G,out_dim", [((8, 7, 9), (17, 13, 10)), ((4, 4, 4), (1, 9, 30)),
                                       ((6, 5, 40), (20, 18, 52)), ((8, 8, 8), (64, 48, 40))])
def test_bspline_f32_parity_mode_within_rounding_of_definition(G, out_dim):
    """The FP32 parity-mode field differs from the FP64 definition only by
    rounding (u = 2^-24): each of the 64 terms carries at most about 20u
    relative error from the basis and the fmaf chains, and the weights sum to
    1, so 20u max|C|; the cell coordinate s = p * inv_h is off by at most 2u s
    <= 2u (G - 3) per axis, and |du/ds| <= 2 max|C| per axis."""
    rng = np.random.default_rng(sum(G) + sum(out_dim))
    C = (5.0 * rng.standard_normal((3,) + G)).astype(np.float32)
    u32 = oracle.bspline_upsample_f32(C, out_dim)
    u64 = oracle.bspline_upsample(C.astype(np.float64), out_dim)
    assert u32.dtype == np.float32 and u32.shape == u64.shape
    bound = 2.0 ** -24 * (20 + 12 * (max(G) - 3)) * np.abs(C).max()
    assert np.abs(u32 - u64).max() <= bound


def test_bspline_adjoint_identity():
    rng = np.random.default_rng(19)
    G = (8, 8, 8)
    out_dim = (19, 14, 23)
    C = rng.standard_normal((3,) + G)
    g = rng.standard_normal((3,) + out_dim)
    lhs = np.vdot(oracle.bspline_upsample(C, out_dim), g)
    rhs = np.vdot(C, oracle.bspline_adjoint(g, G))
    assert lhs == pytest.approx(rhs, rel=1e-12)


# --------------------------------------------------------------------------
# C-P12, C-P13: Philox words, uniforms, Box-Muller Gaussians
# --------------------------------------------------------------------------

def _rocrand_driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host driver")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_host")
    subprocess.run([hipcc, "-O1", "-x", "c++", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    os.path.join(HERE, "rocrand_philox_host.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand_host_engine(tmp_path_factory):
    exe = _rocrand_driver(tmp_path_factory)
    rng = np.random.default_rng(20)
    cases = [(0, 0, 0), (2 ** 64 - 1, 2 ** 32 - 1, 4 * (2 ** 40 + 3)), (20181129, 3, 4 * 12345)]
    for _ in range(40):
        cases.append((int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 32)),
                      4 * int(rng.integers(0, 2 ** 50))))
    inp = "".join(f"{s} {v} {o}\n" for s, v, o in cases)
    res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    words = np.array(res, dtype=np.uint64).reshape(-1, 4).astype(np.uint32)
    for (seed, vol, off), w in zip(cases, words):
        ours = oracle.noise_words(seed, vol, off // 4, 1)[0]
        assert np.array_equal(ours, w), (seed, vol, off)


def test_uniform_mapping():
    for w, expect in [(0, 0.5 * 2 ** -23), (0xFFFFFFFF, 1 - 0.5 * 2 ** -23), (1 << 31, 0.5 + 0.5 * 2 ** -23),
                      (511, 0.5 * 2 ** -23), (512, 1.5 * 2 ** -23)]:
        u = oracle.uniform(w)
        assert u == expect
        assert float(np.float32(u)) == u


def test_gaussian_statistics():
    n = 1 << 21
    z = oracle.gauss(seed=987654321, vol=3, v0=0, n=n)
    assert np.all(np.abs(z) <= np.sqrt(48 * np.log(2)) + 1e-12)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    k = scipy.stats.kurtosis(z, fisher=False)
    assert abs(k - 3) < 5 * np.sqrt(24 / n)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a pair are uncorrelated, and groups differ per volume
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / np.sqrt(n / 2)
    z2 = oracle.gauss(seed=987654321, vol=4, v0=0, n=4096)
    assert not np.allclose(z[:4096], z2)


def test_gaussian_box_muller_pair_structure():
    # r^2 = z_even^2 + z_odd^2 = -2 ln U(w_even), angle = 2 pi U(w_odd)
    w = oracle.noise_words(42, 7, 0, 64)
    z = oracle.gauss(42, 7, 0, 256).reshape(64, 2, 2)
    for g in range(64):
        for pair in range(2):
            ur = oracle.uniform(int(w[g, 2 * pair]))
            ut = oracle.uniform(int(w[g, 2 * pair + 1]))
            zc, zs = z[g, pair]
            assert zc * zc + zs * zs == pytest.approx(-2 * np.log(ur), rel=1e-12)
            assert np.arctan2(zs, zc) % (2 * np.pi) == pytest.approx(2 * np.pi * ut, rel=1e-9, abs=1e-12)


def test_box_muller_on_words_matches_noise_groups():
    w = oracle.noise_words(7, 3, 100, 32)
    z = oracle.gauss(7, 3, 400, 128)
    np.testing.assert_array_equal(oracle.box_muller(w.ravel()), z)


# --------------------------------------------------------------------------
# Photometric chain: paper's window examples, gain/offset/gamma, noise
# --------------------------------------------------------------------------

def _golden_windows():
    rows = []
    with open(os.path.join(HERE, "golden", "window_examples.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(float(t) for t in line.split()))
    return rows


def test_window_examples_from_paper():
    rows = _golden_windows()
    assert len(rows) >= 10
    for a, b, hu, expect in rows:
        ph = PhotoParams(win_lo=a, win_hi=b, window=True, gamma=1.0)
        got = oracle.photometric(np.array([hu]), ph)[0]
        assert got == pytest.approx(expect, abs=1e-15)


def test_gain_offset_gamma_closed_forms():
    V = np.linspace(-1500, 1800, 331)
    ph = PhotoParams(gain=1.0625, offset=-12.5, sigma=0.0, window=False)
    np.testing.assert_array_equal(oracle.photometric(V, ph), 1.0625 * V - 12.5)
    # window then gamma: values whose windowed t is a power of two, with
    # exponents exact in FP32, have exact closed forms t^gamma
    cases = [  # (v in HU, gamma, t^gamma) on the window [-1000, 1000]
        (-500.0, 0.5, 0.5),          # t = 1/4
        (-875.0, 1.25, 1.0 / 32),    # t = 1/16
        (125.0, 0.5, 0.75),          # t = 9/16
        (-500.0, 1.5, 0.125),        # t = 1/4
        (-1000.0 + 2000.0 / 1024, 0.8, 2.0 ** (-10 * float(np.float32(0.8)))),
        (-1000.0, 0.8, 0.0),         # t = 0: 0^gamma = 0
        (-2500.0, 1.25, 0.0),        # below the window
        (1000.0, 0.8, 1.0),          # t = 1
        (4000.0, 0.5, 1.0),          # above the window
    ]
    for v, gam, expect in cases:
        ph = PhotoParams(gain=1.0, offset=0.0, win_lo=-1000, win_hi=1000, gamma=gam, window=True)
        got = oracle.photometric(np.array([v]), ph)[0]
        assert got == pytest.approx(expect, rel=1e-15, abs=0), (v, gam)
    # gain and offset act before the window: V = 200 with gain 1/2 and offset
    # -600 is v = -500, t = 1/4
    ph = PhotoParams(gain=0.5, offset=-600.0, win_lo=-1000, win_hi=1000, gamma=0.5, window=True)
    assert oracle.photometric(np.array([200.0]), ph)[0] == 0.5


def test_noise_is_additive_gaussian_per_voxel():
    n = 1 << 16
    V = np.zeros(n)
    ph = PhotoParams(sigma=10.0, seed=555, volume_id=2, window=False)
    out = oracle.photometric(V, ph)
    np.testing.assert_allclose(out, 10.0 * oracle.gauss(555, 2, 0, n), rtol=1e-15)
    assert abs(out.std() - 10.0) < 0.2


def test_fused_photometric_equals_unfused_oracle():
    rng = np.random.default_rng(21)
    dims = (9, 8, 12)
    img, _ = phantom_pair(dims, seed=61)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    ph = PhotoParams(gain=1.05, offset=7.0, sigma=10.0, win_lo=-1000, win_hi=1000, gamma=0.9,
                     window=True, seed=99, volume_id=1)
    fused, _ = oracle.warp(img, M, dims, photo=ph)
    plain, _ = oracle.warp(img, M, dims)
    np.testing.assert_array_equal(fused, oracle.photometric(plain, ph))


# ---------------------------------------------------------------------------
# Random occlusion (occlusion paragraph and its I_occ equation)
# ---------------------------------------------------------------------------

def _occ_case(lo, hi, **kw):
    rng = np.random.default_rng(31)
    dims = (10, 9, 14)
    img, lbl = phantom_pair(dims, seed=71)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    M = oracle.affine_matrix(prm, dims, dims)
    ph = PhotoParams(occlude=True, occ_lo=lo, occ_hi=hi, **kw)
    return img, lbl, M, dims, ph


@pytest.mark.parametrize("lo,hi,slab", [(3.0, 7.0, [3, 4, 5, 6, 7]), (2.5, 5.5, [3, 4, 5]),
                                        (-4.0, 0.0, [0]), (12.25, 30.0, [13]),
                                        (5.2, 5.8, []), (-9.0, -1.0, [])])
def test_occluded_slab_is_zero_then_photometrics(lo, hi, slab):
    """Voxels with occ_lo <= z <= occ_hi (closed) take I_occ = 0 before the
    photometric chain (here gain/offset only: exactly the offset); the rest
    and every label equal the unoccluded warp."""
    img, lbl, M, dims, ph = _occ_case(lo, hi, gain=1.5, offset=-12.0, window=False)
    out, lout = oracle.warp(img, M, dims, lbl=lbl, photo=ph)
    ref_ph = PhotoParams(gain=1.5, offset=-12.0, window=False)
    ref, lref = oracle.warp(img, M, dims, lbl=lbl, photo=ref_ph)
    z = np.arange(dims[2])
    occ = np.isin(z, slab)
    assert np.all(out[:, :, occ] == -12.0)
    np.testing.assert_array_equal(out[:, :, ~occ], ref[:, :, ~occ])
    np.testing.assert_array_equal(lout, lref)


def test_occluded_voxels_still_get_noise_and_window():
    """The noise equation adds n to I_occ, so occluded voxels are
    window(offset + sigma n(v)) with the voxel's own Gaussian."""
    img, lbl, M, dims, ph = _occ_case(4.0, 9.0, gain=1.1, offset=20.0, sigma=25.0, win_lo=-200,
                                      win_hi=300, gamma=1.0, window=True, seed=7, volume_id=3)
    out, _ = oracle.warp(img, M, dims, photo=ph)
    n = oracle.gauss(7, 3, 0, int(np.prod(dims))).reshape(dims)
    f32 = lambda v: float(np.float32(v))
    expect = np.clip((f32(20.0) + f32(25.0) * n - f32(-200)) / (f32(300) - f32(-200)), 0, 1)
    np.testing.assert_allclose(out[:, :, 4:10], expect[:, :, 4:10], rtol=1e-12, atol=1e-15)


def test_occlusion_fused_equals_unfused():
    img, lbl, M, dims, ph = _occ_case(1.0, 6.5, gain=0.95, offset=3.0, sigma=10.0, window=True,
                                      win_lo=-1000, win_hi=1000, gamma=0.8, seed=5, volume_id=2)
    fused, _ = oracle.warp(img, M, dims, photo=ph)
    plain, _ = oracle.warp(img, M, dims)
    np.testing.assert_array_equal(fused, oracle.photometric(plain, ph))


def test_occlusion_draw_covers_every_slice_equally():
    """Start ~ U[-delta_max, z_max], height ~ U[0, delta_max]: every z in
    [0, z_max] is occluded with probability (delta_max / 2) / (z_max + delta_max)."""
    from synth import draw_occlusion
    rng = np.random.default_rng(2024)
    dmax, zmax, n = 16.0, 63, 200000
    draws = np.array([draw_occlusion(rng, dmax, zmax) for _ in range(n)])
    z = np.arange(zmax + 1)
    freq = ((draws[:, :1] <= z) & (z <= draws[:, 1:])).mean(0)
    p = (dmax / 2) / (zmax + dmax)
    assert np.abs(freq - p).max() < 5 * np.sqrt(p * (1 - p) / n)


# ---------------------------------------------------------------------------
# Resampling pre-step: Gaussian smoothing (Pre- and post-processing section)
# ---------------------------------------------------------------------------

def test_resample_sigma_formula_examples():
    """sigma_k = max(r / u_k - 1, 0) / 3: no smoothing when the target is not
    coarser, 1 voxel when the target is 4x coarser."""
    np.testing.assert_allclose(oracle.resample_sigma([3.0, 0.75, 6.0], 3.0), [0.0, 1.0, 0.0])
    np.testing.assert_allclose(oracle.resample_sigma([0.5, 1.5, 2.5], 3.0),
                               [5.0 / 3.0, 1.0 / 3.0, 0.2 / 3.0], rtol=1e-15)


def test_gaussian_smooth_zero_sigma_is_identity_and_constants_stay():
    rng = np.random.default_rng(3)
    v = rng.normal(0, 100, (9, 7, 11))
    np.testing.assert_array_equal(oracle.gaussian_smooth(v, [0, 0, 0]), v)
    c = np.full((8, 9, 10), -321.5)
    np.testing.assert_allclose(oracle.gaussian_smooth(c, [2.0, 1.3, 0.7]), c, rtol=1e-14)


def test_gaussian_smooth_impulse_is_normalised_kernel():
    """An interior impulse spreads into the outer product of the normalised
    1-D kernels exp(-d^2 / sigma^2), |d| <= floor(3 sigma / sqrt 2 + 0.5)."""
    sig = [1.7, 0.9, 2.6]
    v = np.zeros((21, 17, 25))
    v[10, 8, 12] = 1.0
    out = oracle.gaussian_smooth(v, sig)
    ks = []
    for s_ in sig:
        R = int(np.floor(3 * s_ / np.sqrt(2) + 0.5))
        d = np.arange(-R, R + 1)
        k = np.exp(-d.astype(float) ** 2 / s_ ** 2)
        ks.append(k / k.sum())
    ref = np.zeros_like(v)
    Rs = [(len(k) - 1) // 2 for k in ks]
    ref[10 - Rs[0]:10 + Rs[0] + 1, 8 - Rs[1]:8 + Rs[1] + 1, 12 - Rs[2]:12 + Rs[2] + 1] = \
        np.einsum("i,j,k->ijk", *ks)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("sig", [(1.2, 0.0, 2.2), (0.45, 3.1, 0.8)])
def test_gaussian_smooth_matches_scipy_nearest(sig):
    """exp(-d^2/sigma^2) is a Gaussian of standard deviation sigma / sqrt 2;
    SciPy's gaussian_filter with that deviation, truncate=3 (the same radius)
    and mode 'nearest' (edge repeat) computes the same sums."""
    from scipy import ndimage
    rng = np.random.default_rng(17)
    v = rng.normal(0, 300, (14, 12, 19))
    sd = [s_ / np.sqrt(2) for s_ in sig]
    ref = v.copy()
    for ax, s_ in enumerate(sd):
        if s_ > 0:
            ref = ndimage.gaussian_filter1d(ref, s_, axis=ax, mode="nearest", truncate=3.0)
    np.testing.assert_allclose(oracle.gaussian_smooth(v, sig), ref, rtol=1e-12, atol=1e-10)
