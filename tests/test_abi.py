"""The C ABI of libctaug.so without a GPU: the library loads, exports every
entry point include/ctaug.h declares, host-side calls compute what the
header says, and argument validation rejects bad input before anything is
enqueued (every case here returns before the first HIP call)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1811_11226_amd import _lib
from synth.draws import AugmentRanges, draw_affine_params

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "ctaug.h")

OK, EINVAL, EDTYPE, ESHAPE, EWORKSPACE = 0, 1, 2, 3, 4
F32, I16, I8 = _lib.CTAUG_F32, _lib.CTAUG_I16, _lib.CTAUG_I8
FAKE = 0x1000          # never dereferenced: every call below fails validation first


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libctaug.so is not built")
    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|(?:int|size_t|ctaug_status)\s+)"
                                 r"(ctaug_\w+)\s*\(", text, flags=re.M)))


def vol(dims, dtype=F32, data=FAKE, reserved=0, stride=None):
    v = _lib.Vol()
    v.data = data
    v.dtype = dtype
    v.reserved = reserved
    for i in range(3):
        v.dim[i] = dims[i]
        v.stride[i] = 0 if stride is None else stride[i]
    return v


def mat(M=None):
    M = np.eye(3, 4, dtype=np.float32).ravel() if M is None else np.asarray(M, np.float32)
    return (ctypes.c_float * 12)(*[float(x) for x in M])


def photo(**kw):
    p = _lib.Photo()
    p.gain, p.offset, p.sigma = 1.0, 0.0, 0.0
    p.win_lo, p.win_hi, p.gamma = -1000.0, 1000.0, 1.0
    p.flags, p.volume_id, p.seed = 0, 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def warp(L, img, lbl, M, fill, lfill, ph, out, lout):
    r = ctypes.byref
    return L.ctaug_warp_affine(r(img) if img is not None else None,
                               r(lbl) if lbl is not None else None, M, fill, lfill,
                               r(ph) if ph is not None else None,
                               r(out) if out is not None else None,
                               r(lout) if lout is not None else None, None)


# -- symbols ----------------------------------------------------------------

def test_header_declares_entry_points():
    names = declared_symbols()
    assert len(names) >= 20
    assert "ctaug_warp_affine" in names and "ctaug_batch_plan_create" in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"
    assert set(_lib.SIGNATURES) == set(declared_symbols())


def test_status_strings_and_version(L):
    for s in range(7):
        assert L.ctaug_status_string(s)
    assert L.ctaug_status_string(0) == b"ok"
    assert L.ctaug_status_string(99) == b"unknown status"
    assert L.ctaug_version() >= 10000


# -- transform composition (host) ---------------------------------------------

def _params(prm):
    p = _lib.AffineParams()
    fields = [("rot", 0, 3), ("scale", 3, 3), ("shear", 6, 3), ("reflect", 9, 3),
              ("generic", 12, 9), ("disp", 21, 3), ("crop", 24, 3)]
    for name, off, n in fields:
        arr = getattr(p, name)
        for i in range(n):
            arr[i] = float(prm[off + i])
    return p


def lib_affine(L, prm, in_dim, out_dim):
    p = _params(prm)
    idim = (ctypes.c_int64 * 3)(*in_dim)
    odim = (ctypes.c_int64 * 3)(*out_dim)
    M64, M32 = (ctypes.c_double * 12)(), (ctypes.c_float * 12)()
    st = L.ctaug_affine_matrix(ctypes.byref(p), idim, odim, M64, M32)
    return st, np.array(M64[:]), np.array(M32[:], dtype=np.float32)


@pytest.mark.parametrize("seed", range(12))
def test_affine_matrix_matches_oracle(L, seed):
    rng = np.random.Generator(np.random.PCG64(900 + seed))
    ranges = AugmentRanges(rot_deg=(180.0, 180.0, 180.0), shear=(0.3, 0.3, 0.3),
                           reflect_prob=(0.5, 0.5, 0.5), generic=0.2, isotropic=bool(seed % 2))
    in_dim = tuple(int(v) for v in rng.integers(1, 300, 3))
    out_dim = tuple(int(v) for v in rng.integers(1, 300, 3))
    prm = draw_affine_params(rng, ranges, in_dim, out_dim)
    st, M64, M32 = lib_affine(L, prm, in_dim, out_dim)
    assert st == OK
    ref = oracle.affine_matrix(prm, in_dim, out_dim)
    # both sides compose in FP64 with different association: agree to a few ulps
    scale = np.abs(ref).max() + 1.0
    np.testing.assert_allclose(M64, ref, rtol=0, atol=64 * np.finfo(np.float64).eps * scale)
    np.testing.assert_array_equal(M32, M64.astype(np.float32))


def test_affine_matrix_identity_maps_centre_to_centre(L):
    prm = np.zeros(27)
    prm[3:6] = 1.0
    prm[12:21] = np.eye(3).ravel()
    st, M64, _ = lib_affine(L, prm, (11, 20, 7), (5, 8, 9))
    assert st == OK
    A, b = M64.reshape(3, 4)[:, :3], M64.reshape(3, 4)[:, 3]
    np.testing.assert_array_equal(A, np.eye(3))
    np.testing.assert_allclose(A @ np.array([2.0, 3.5, 4.0]) + b, [5.0, 9.5, 3.0])


def test_affine_matrix_errors(L):
    prm = np.zeros(27)
    prm[3:6] = 1.0
    p = _params(prm)
    d = (ctypes.c_int64 * 3)(4, 4, 4)
    neg = (ctypes.c_int64 * 3)(4, -1, 4)
    M64 = (ctypes.c_double * 12)()
    assert L.ctaug_affine_matrix(None, d, d, M64, None) == EINVAL
    assert L.ctaug_affine_matrix(ctypes.byref(p), d, d, None, None) == EINVAL
    assert L.ctaug_affine_matrix(ctypes.byref(p), neg, d, M64, None) == ESHAPE
    p.rot[1] = math.nan
    assert L.ctaug_affine_matrix(ctypes.byref(p), d, d, M64, None) == EINVAL
    p.rot[1] = 0.0
    p.crop[2] = math.inf
    assert L.ctaug_affine_matrix(ctypes.byref(p), d, d, M64, None) == EINVAL


# -- forward warp validation --------------------------------------------------

def test_warp_rejects_bad_arguments(L):
    img, out = vol((8, 8, 8), I16), vol((4, 4, 4))
    lbl, lout = vol((8, 8, 8), I8), vol((4, 4, 4), I8)
    M, ph = mat(), photo()
    assert warp(L, None, None, M, 0.0, 0, None, out, None) == EINVAL
    assert warp(L, img, None, None, 0.0, 0, None, out, None) == EINVAL
    assert warp(L, vol((8, 8, 8), I16, reserved=1), None, M, 0.0, 0, None, out, None) == EINVAL
    assert warp(L, vol((8, 8, 8), I8), None, M, 0.0, 0, None, out, None) == EDTYPE
    assert warp(L, vol((8, 8, 8), 7), None, M, 0.0, 0, None, out, None) == EDTYPE
    assert warp(L, img, None, M, 0.0, 0, None, vol((4, 4, 4), I16), None) == EDTYPE
    assert warp(L, vol((8, -1, 8), I16), None, M, 0.0, 0, None, out, None) == ESHAPE
    assert warp(L, vol((1 << 16, 1 << 16, 1), I16), None, M, 0.0, 0, None, out, None) == ESHAPE
    assert warp(L, vol((1 << 10, 1 << 10, 1 << 10), F32), None, M, 0.0, 0, None, out,
                None) == ESHAPE
    assert warp(L, vol((8, 8, 8), I16, data=None), None, M, 0.0, 0, None, out, None) == EINVAL
    # labels: dtype, dims, missing output
    assert warp(L, img, vol((8, 8, 8), F32), M, 0.0, 0, None, out, lout) == EDTYPE
    assert warp(L, img, vol((8, 8, 7), I8), M, 0.0, 0, None, out, lout) == ESHAPE
    assert warp(L, img, lbl, M, 0.0, 0, None, out, None) == EINVAL
    assert warp(L, img, lbl, M, 0.0, 0, None, out, vol((4, 4, 5), I8)) == ESHAPE
    # parameters
    bad = np.eye(3, 4, dtype=np.float32).ravel()
    bad[5] = np.inf
    assert warp(L, img, None, mat(bad), 0.0, 0, None, out, None) == EINVAL
    assert warp(L, img, None, M, math.nan, 0, None, out, None) == EINVAL
    assert warp(L, img, lbl, M, 0.0, 128, None, out, lout) == EINVAL
    assert warp(L, img, lbl, M, 0.0, -129, None, out, lout) == EINVAL


# -- layouts and the kernels' 24-bit offset arithmetic --------------------------

EMPTY_OUT = dict(dims=(0, 4, 4), data=None)


def test_gather_offsets_beyond_24_bits_are_rejected(L):
    """Input offsets are (ix ry + iy) sy + iz with 24-bit multiplies: shapes
    whose row count (X-1) ry + Y exceeds 2^24, or whose row pitch reaches
    2^24, are refused before anything runs (an empty output makes an accepted
    call a no-op, so acceptance is visible without a GPU)."""
    out = vol(**EMPTY_OUT)
    M = mat()
    for dims in [(2, 1 << 24, 4), (8192, 4096, 2), (1, 1, 1 << 24), (4097, 4096, 1),
                 (2, (1 << 23) + 1, 1)]:
        assert warp(L, vol(dims, I16), None, M, 0.0, 0, None, out, None) == ESHAPE, dims
        lbl, lout = vol(dims, I8), vol((0, 4, 4), I8, data=None)
        assert warp(L, vol(dims, I16), lbl, M, 0.0, 0, None, out, lout) == ESHAPE, dims
    # just inside: X*Y = 2^24 rows, row pitch 2^24 - 1
    for dims in [(4096, 4096, 1), (1 << 12, 1 << 12, 2), (1, 1, (1 << 24) - 1), (1, 1 << 24, 1)]:
        assert warp(L, vol(dims, I16), None, M, 0.0, 0, None, out, None) == OK, dims
    # a strided view: its parent's rows count (here 2^24 + 256 rows)
    par = (1 << 12, (1 << 12) + 1, 4)
    st = (par[1] * par[2], par[2], 1)
    assert warp(L, vol((4096, 4096, 4), I16, stride=st), None, M, 0.0, 0, None, out,
                None) == ESHAPE
    assert warp(L, vol((4095, 4096, 4), I16, stride=st), None, M, 0.0, 0, None, out,
                None) == OK
    # the adjoints read the same image
    r = ctypes.byref
    big = vol((8192, 4096, 2), I16)
    assert L.ctaug_warp_affine_backward(r(big), M, 0.0, None, r(vol((0, 4, 4), data=None)), None,
                                        None, None, 0, None) == ESHAPE


def test_strided_layouts(L):
    """Strided views are accepted for gathered inputs only, with z contiguous
    and the x stride a whole number of y rows."""
    out, M = vol(**EMPTY_OUT), mat()
    ok = [(40 * 30, 30, 1), (40 * 30 * 3, 30, 1), (0, 0, 0), (8 * 8, 8, 1)]
    for st in ok:
        assert warp(L, vol((8, 8, 8), I16, stride=st), None, M, 0.0, 0, None, out, None) == OK, st
    bad = [(64, 8, 2),          # z not contiguous
           (64, 7, 1),          # row pitch below Z
           (60, 8, 1),          # x stride not a whole number of rows
           (56, 8, 1),          # fewer rows per plane than Y
           (64, 0, 1), (-64, 8, 1), (0, 8, 1)]
    for st in bad:
        assert warp(L, vol((8, 8, 8), I16, stride=st), None, M, 0.0, 0, None, out,
                    None) == ESHAPE, st
    # labels must share the image's layout
    img = vol((8, 8, 8), I16, stride=(40 * 30, 30, 1))
    lout = vol((0, 4, 4), I8, data=None)
    assert warp(L, img, vol((8, 8, 8), I8, stride=(40 * 30, 30, 1)), M, 0.0, 0, None, out,
                lout) == OK
    assert warp(L, img, vol((8, 8, 8), I8), M, 0.0, 0, None, out, lout) == ESHAPE
    # outputs must be dense
    assert warp(L, vol((8, 8, 8), I16), None, M, 0.0, 0, None,
                vol((4, 4, 4), stride=(40, 10, 1)), None) == ESHAPE
    # an FP32 input's byte extent must fit a 32-bit buffer range
    assert warp(L, vol((2, 2, 2), F32, stride=(1 << 30, 1 << 15, 1)), None, M, 0.0, 0, None,
                out, None) == ESHAPE
    assert warp(L, vol((2, 2, 2), I16, stride=(1 << 30, 1 << 15, 1)), None, M, 0.0, 0, None,
                out, None) == OK
    # dense-only arguments elsewhere
    ph = photo()
    assert L.ctaug_photometric_noise(ctypes.byref(vol((4, 4, 4), stride=(40, 10, 1))),
                                     ctypes.byref(ph), None) == ESHAPE


@pytest.mark.parametrize("kw", [dict(sigma=-1.0), dict(gamma=0.0), dict(gain=math.nan),
                                dict(flags=4), dict(flags=1, win_lo=5.0, win_hi=5.0),
                                dict(offset=math.inf), dict(flags=2, occ_lo=math.nan),
                                dict(flags=3, occ_hi=math.inf)])
def test_warp_rejects_bad_photometrics(L, kw):
    ph = photo(**kw)
    assert warp(L, vol((8, 8, 8), I16), None, mat(), 0.0, 0, ph, vol((4, 4, 4)), None) == EINVAL
    assert L.ctaug_photometric_noise(ctypes.byref(vol((4, 4, 4))), ctypes.byref(ph), None) == EINVAL


def test_empty_volumes_are_no_ops(L):
    # a zero dimension makes a call return OK without touching the device
    out = vol((0, 4, 4), data=None)
    assert warp(L, vol((8, 8, 8), I16), None, mat(), 0.0, 0, None, out, None) == OK
    assert warp(L, vol((0, 8, 8), I16, data=None), None, mat(), 0.0, 0, None,
                vol((0, 2, 2), data=None), None) == OK
    assert L.ctaug_photometric_noise(ctypes.byref(vol((3, 0, 3), data=None)),
                                     ctypes.byref(photo()), None) == OK
    assert L.ctaug_noise(1, 0, 0, 0, None, None, None) == OK
    assert L.ctaug_box_muller(None, 0, None, None) == OK
    assert L.ctaug_copy(None, None, 0, None) == OK


def test_labels_only_warp_validation(L):
    r = ctypes.byref
    lin, lout = vol((8, 8, 8), I8), vol((4, 4, 4), I8)
    assert L.ctaug_warp_labels(None, mat(), 0, r(lout), None) == EINVAL
    assert L.ctaug_warp_labels(r(lin), mat(), 0, None, None) == EINVAL
    assert L.ctaug_warp_labels(r(lin), None, 0, r(lout), None) == EINVAL
    assert L.ctaug_warp_labels(r(lin), mat([math.inf] + [0.0] * 11), 0, r(lout), None) == EINVAL
    for lf in (-129, 128):
        assert L.ctaug_warp_labels(r(lin), mat(), lf, r(lout), None) == EINVAL
    assert L.ctaug_warp_labels(r(vol((8, 8, 8), I16)), mat(), 0, r(lout), None) == EDTYPE
    assert L.ctaug_warp_labels(r(lin), mat(), 0, r(vol((4, 4, 4))), None) == EDTYPE
    assert L.ctaug_warp_labels(r(lin), mat(), 0, r(vol((4, -1, 4), I8)), None) == ESHAPE
    assert L.ctaug_warp_labels(r(vol((8, 8, 8), I8, reserved=1)), mat(), 0, r(lout), None) == EINVAL
    # a strided input is accepted (a crop view); a strided output is not
    crop = vol((4, 4, 4), I8, stride=(64, 8, 1))
    assert L.ctaug_warp_labels(r(crop), mat(), 0, r(vol((0, 4, 4), I8, data=None)), None) == OK
    assert L.ctaug_warp_labels(r(lin), mat(), 0, r(vol((4, 4, 4), I8, stride=(64, 8, 1))),
                               None) == ESHAPE
    # rows beyond the 24-bit gather limit
    assert L.ctaug_warp_labels(r(vol((2, 1 << 24, 4), I8)), mat(), 0, r(lout), None) == ESHAPE
    # an empty output is a no-op
    assert L.ctaug_warp_labels(r(lin), mat(), 0, r(vol((4, 0, 4), I8, data=None)), None) == OK


def test_displacement_and_noise_validation(L):
    img, out = ctypes.byref(vol((8, 8, 8), I16)), ctypes.byref(vol((4, 4, 4)))
    assert L.ctaug_warp_displacement(img, None, mat(), None, 0.0, 0, None, out, None,
                                     None) == EINVAL
    assert L.ctaug_photometric_noise(ctypes.byref(vol((4, 4, 4))), None, None) == EINVAL
    assert L.ctaug_photometric_noise(ctypes.byref(vol((4, 4, 4), I16)), ctypes.byref(photo()),
                                     None) == EDTYPE
    assert L.ctaug_noise(1, 0, 0, -1, FAKE, None, None) == EINVAL
    assert L.ctaug_noise(1, 0, (1 << 64) - 4, 8, FAKE, None, None) == EINVAL
    assert L.ctaug_box_muller(None, 3, FAKE, None) == EINVAL
    assert L.ctaug_box_muller(FAKE, -1, FAKE, None) == EINVAL
    assert L.ctaug_copy(None, FAKE, 16, None) == EINVAL


# -- adjoints -----------------------------------------------------------------

def test_backward_workspace_and_validation(L):
    d = (ctypes.c_int64 * 3)(64, 64, 64)
    ws = L.ctaug_warp_backward_workspace(d)
    assert ws > 0 and ws % (12 * 8) == 0
    assert L.ctaug_warp_backward_workspace((ctypes.c_int64 * 3)(4, -2, 4)) == 0
    assert L.ctaug_warp_backward_workspace((ctypes.c_int64 * 3)(0, 4, 4)) == 0
    img, g = vol((8, 8, 8)), vol((64, 64, 64))
    gM = FAKE
    r = ctypes.byref
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, None, r(g), None, gM, None, 0,
                                        None) == EWORKSPACE
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, None, r(g), None, gM, FAKE, ws - 8,
                                        None) == EWORKSPACE
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, None, r(g), r(vol((8, 8, 9))), None, None,
                                        0, None) == ESHAPE
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, None, r(vol((64, 64, 64), I16)), None, gM,
                                        FAKE, ws, None) == EDTYPE
    assert L.ctaug_warp_displacement_backward(r(img), mat(), None, 0.0, None, r(g), None, gM, None,
                                              FAKE, ws, None) == EINVAL
    # the photometric adjoint: the windowed chain is not differentiated, and
    # parameters are validated as in the forward
    out0 = vol((0, 4, 4), data=None)
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, r(photo(flags=1)), r(out0), None,
                                        None, None, 0, None) == EINVAL
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, r(photo(gain=math.nan)), r(out0),
                                        None, None, None, 0, None) == EINVAL
    assert L.ctaug_warp_affine_backward(r(img), mat(), 0.0, r(photo(flags=2, occ_lo=1.0,
                                                                     occ_hi=3.0)),
                                        r(out0), None, None, None, 0, None) == OK


def test_bspline_validation(L):
    od = (ctypes.c_int64 * 3)(32, 32, 32)
    for G in [(3, 8, 8), (8, 65, 8), (8, 8, -1)]:
        g = (ctypes.c_int64 * 3)(*G)
        assert L.ctaug_bspline_upsample(FAKE, g, od, FAKE, None) == ESHAPE
        assert L.ctaug_bspline_adjoint_workspace(od, g) == 0
    g = (ctypes.c_int64 * 3)(8, 8, 8)
    assert L.ctaug_bspline_upsample(None, g, od, FAKE, None) == EINVAL
    assert L.ctaug_bspline_upsample(FAKE, None, od, FAKE, None) == EINVAL
    need = L.ctaug_bspline_adjoint_workspace(od, g)
    assert need > 0
    assert L.ctaug_bspline_upsample_adjoint(FAKE, od, g, FAKE, FAKE, need - 1, None) == EWORKSPACE
    assert L.ctaug_bspline_upsample_adjoint(FAKE, od, g, None, FAKE, need, None) == EINVAL


def test_fused_bspline_warp_validation(L):
    r = ctypes.byref
    img, out = vol((8, 8, 8), I16), vol((32, 32, 32))
    g = (ctypes.c_int64 * 3)(8, 8, 8)

    def call(ctrl, G, out_vol=out, M=None):
        return L.ctaug_warp_bspline(r(img), None, mat() if M is None else M, ctrl, G, 0.0, 0,
                                    None, r(out_vol), None, None)

    assert call(None, g) == EINVAL                 # no control grid
    assert call(FAKE, None) == EINVAL              # no grid dims
    for G in [(3, 8, 8), (8, 65, 8), (8, 8, 0)]:
        assert call(FAKE, (ctypes.c_int64 * 3)(*G)) == ESHAPE
    bad = mat()
    bad[3] = float("nan")
    assert call(FAKE, g, M=bad) == EINVAL
    assert call(FAKE, g, out_vol=vol((32, 32, 32), I16)) == EDTYPE
    # an empty output needs no control grid and touches nothing
    assert call(None, g, out_vol=vol((0, 32, 32), data=None)) == OK


def test_fused_bspline_backward_workspace_and_validation(L):
    r = ctypes.byref
    od = (ctypes.c_int64 * 3)(64, 64, 64)
    g8 = (ctypes.c_int64 * 3)(8, 8, 8)
    rows = L.ctaug_warp_backward_workspace(od) // 96
    m = -(-rows * 96 // 256) * 256
    # 8^3 grid over 64^3: the fused route, one row of control gradients per workgroup
    assert L.ctaug_warp_bspline_backward_workspace(od, g8) == \
        m + (rows + min(rows, 64)) * 3 * 512 * 8
    # controls closer than 2 voxels along z: the dense route (field, its gradient,
    # the B-spline adjoint's workspace)
    gz = (ctypes.c_int64 * 3)(8, 8, 60)
    dense = L.ctaug_warp_bspline_backward_workspace(od, gz)
    field = -(-3 * 64 ** 3 * 4 // 256) * 256
    assert dense == m + 2 * field + L.ctaug_bspline_adjoint_workspace(od, gz)
    assert L.ctaug_warp_bspline_backward_workspace(od, (ctypes.c_int64 * 3)(3, 8, 8)) == 0
    assert L.ctaug_warp_bspline_backward_workspace(None, g8) == 0
    img, g = vol((8, 8, 8)), vol((64, 64, 64))
    need = L.ctaug_warp_bspline_backward_workspace(od, g8)

    def call(ctrl=FAKE, G=g8, gimg=None, gM=FAKE, gc=FAKE, ws=FAKE, nbytes=need, gout=g):
        return L.ctaug_warp_bspline_backward(r(img), mat(), ctrl, G, 0.0, None, r(gout),
                                             r(gimg) if gimg is not None else None, gM, gc, ws,
                                             nbytes, None)

    assert call(ws=None) == EWORKSPACE
    assert call(nbytes=need - 8) == EWORKSPACE
    assert call(G=None) == EINVAL
    assert call(G=(ctypes.c_int64 * 3)(8, 65, 8)) == ESHAPE
    assert call(ctrl=None) == EINVAL
    assert call(gimg=vol((8, 8, 9))) == ESHAPE
    assert call(gout=vol((64, 64, 64), I16)) == EDTYPE


# -- host-to-device FIFO -------------------------------------------------------

def test_pipeline_validation_before_any_hip_call(L):
    h = ctypes.c_void_p()
    assert L.ctaug_pipeline_create(1, 1 << 20, ctypes.byref(h)) == EINVAL
    assert L.ctaug_pipeline_create(65, 1 << 20, ctypes.byref(h)) == EINVAL
    assert L.ctaug_pipeline_create(2, 0, ctypes.byref(h)) == EINVAL
    assert L.ctaug_pipeline_create(2, 1 << 20, None) == EINVAL
    slot = ctypes.c_void_p()
    assert L.ctaug_pipeline_acquire(None, ctypes.byref(slot)) == EINVAL
    r = ctypes.byref
    assert L.ctaug_pipeline_submit(None, r(vol((4, 4, 4), I16)), None, mat(), 0.0, 0, None,
                                   r(vol((4, 4, 4))), None) == EINVAL
    assert L.ctaug_pipeline_stream(None, ctypes.byref(slot)) == EINVAL
    assert L.ctaug_pipeline_sync(None) == EINVAL
    assert L.ctaug_pipeline_destroy(None) == EINVAL


# -- batch plan ---------------------------------------------------------------

def _job(in_dims=(8, 8, 8), out_dims=(4, 4, 4), dtype=I16):
    j = _lib.Job()
    j.img_in = vol(in_dims, dtype)
    j.lbl_in = vol(in_dims, I8, data=None)
    j.img_out = vol(out_dims)
    j.lbl_out = vol(out_dims, I8, data=None)
    for i, v in enumerate(np.eye(3, 4, dtype=np.float32).ravel()):
        j.M[i] = float(v)
    j.fill = -1000.0
    j.label_fill = 0
    j.photo = photo(flags=_lib.CTAUG_PHOTO_NONE)
    return j


@pytest.mark.parametrize("tile,wg,lds,fmt", [((8, 8, 2), 0, 0, 0), ((3, 8, 8), 0, 0, 0),
                                             ((64, 64, 64), 0, 0, 0), ((8, 8, 8), -1, 0, 0),
                                             ((8, 8, 8), 33, 0, 0), ((8, 8, 8), 0, -2, 0),
                                             ((8, 8, 8), 0, 1 << 20, 0), ((8, 8, 8), 0, 0, 2)])
def test_plan_rejects_bad_tuning(L, tile, wg, lds, fmt):
    t = _lib.Tuning()
    t.tile[:] = tile
    t.wg_per_cu, t.lds_cells, t.lds_format = wg, lds, fmt
    jobs = (_lib.Job * 1)(_job())
    plan = ctypes.c_void_p()
    assert L.ctaug_batch_plan_create(jobs, 1, ctypes.byref(t), ctypes.byref(plan)) == EINVAL
    assert not plan.value


def test_plan_rejects_bad_jobs(L):
    plan = ctypes.c_void_p()
    jobs = (_lib.Job * 2)(_job(), _job(dtype=I8))
    assert L.ctaug_batch_plan_create(jobs, 2, None, ctypes.byref(plan)) == EDTYPE
    jobs = (_lib.Job * 1)(_job())
    assert L.ctaug_batch_plan_create(jobs, 0, None, ctypes.byref(plan)) == EINVAL
    assert L.ctaug_batch_plan_create(None, 1, None, ctypes.byref(plan)) == EINVAL
    assert L.ctaug_batch_plan_create(jobs, 1, None, None) == EINVAL
    bad = _job()
    bad.M[0] = math.nan
    jobs = (_lib.Job * 1)(bad)
    assert L.ctaug_batch_plan_create(jobs, 1, None, ctypes.byref(plan)) == EINVAL
    # B-spline jobs: not mixed with affine ones, and a valid grid
    sp = _job()
    sp.ctrl = FAKE
    sp.grid = (ctypes.c_int64 * 3)(8, 8, 8)
    jobs = (_lib.Job * 2)(sp, _job())
    assert L.ctaug_batch_plan_create(jobs, 2, None, ctypes.byref(plan)) == EINVAL
    sp.grid = (ctypes.c_int64 * 3)(8, 3, 8)
    jobs = (_lib.Job * 1)(sp)
    assert L.ctaug_batch_plan_create(jobs, 1, None, ctypes.byref(plan)) == ESHAPE
    assert not plan.value


def test_plan_calls_reject_null_plan(L):
    t = _lib.Tuning()
    assert L.ctaug_batch_plan_destroy(None) == EINVAL
    assert L.ctaug_batch_plan_get_tuning(None, ctypes.byref(t)) == EINVAL
    assert L.ctaug_batch_plan_launch(None, None) == EINVAL
    assert L.ctaug_batch_plan_run(None, None) == EINVAL
    assert L.ctaug_batch_plan_capture(None, None) == EINVAL
    assert L.ctaug_batch_plan_replay(None, None) == EINVAL
    assert L.ctaug_batch_plan_update(None, None) == EINVAL
    assert L.ctaug_batch_plan_autotune(None, None, 0, 1, None, None, None) == EINVAL


# -- resampling pre-step ----------------------------------------------------------

@pytest.mark.parametrize("spacing,target", [((0.7, 0.7, 2.5), 3.0), ((3.0, 1.0, 0.4), 3.0),
                                            ((5.0, 6.0, 7.0), 3.0)])
def test_resample_sigma_matches_oracle(L, spacing, target):
    sp = (ctypes.c_double * 3)(*spacing)
    out = (ctypes.c_float * 3)()
    assert L.ctaug_resample_sigma(sp, target, out) == OK
    np.testing.assert_array_equal(np.array(out[:], dtype=np.float32),
                                  oracle.resample_sigma(spacing, target).astype(np.float32))


def test_smoothing_validation(L):
    r = ctypes.byref
    sg = (ctypes.c_float * 3)(1.0, 1.0, 0.0)
    a, b = vol((8, 8, 8)), vol((8, 8, 8), data=0x2000)
    assert L.ctaug_resample_sigma(None, 3.0, sg) == EINVAL
    assert L.ctaug_resample_sigma((ctypes.c_double * 3)(1, 0, 1), 3.0, sg) == EINVAL
    assert L.ctaug_resample_sigma((ctypes.c_double * 3)(1, 1, 1), math.nan, sg) == EINVAL
    assert L.ctaug_gaussian_smooth(r(a), r(b), None, None, 0, None) == EINVAL
    assert L.ctaug_gaussian_smooth(r(a), r(vol((8, 8, 9), data=0x2000)), sg, None, 0,
                                   None) == ESHAPE
    assert L.ctaug_gaussian_smooth(r(a), r(vol((8, 8, 8), I16, data=0x2000)), sg, None, 0,
                                   None) == EDTYPE
    assert L.ctaug_gaussian_smooth(r(a), r(a), sg, None, 0, None) == EINVAL          # aliasing
    assert L.ctaug_gaussian_smooth(r(a), r(b), sg, None, 0, None) == EWORKSPACE      # 2 axes
    assert L.ctaug_gaussian_smooth(r(a), r(b), (ctypes.c_float * 3)(-1, 0, 0), None, 0,
                                   None) == EINVAL
    assert L.ctaug_gaussian_smooth(r(a), r(b), (ctypes.c_float * 3)(500, 0, 0), None, 0,
                                   None) == EINVAL                                   # R > 160
    need = L.ctaug_gaussian_smooth_workspace((ctypes.c_int64 * 3)(8, 8, 8))
    assert need == 8 * 8 * 8 * 4


# -- autotune cache (host side) -------------------------------------------------

def test_autotune_cache_save_load_round_trip(L, tmp_path):
    """A saved cache loads back entry for entry; malformed files merge nothing."""
    assert L.ctaug_autotune_cache_clear() == OK
    good = tmp_path / "cache.txt"
    good.write_text("# ctaug autotune cache v1\n"
                    "gfx950 256 1 4 22 3 16 16 16 0 8176 0\n"
                    "gfx950 256 3 3 21 0 8 16 16 2 0 1\n")
    n = ctypes.c_int32(-1)
    assert L.ctaug_autotune_cache_load(str(good).encode(), ctypes.byref(n)) == OK
    assert n.value == 2
    out = tmp_path / "out.txt"
    assert L.ctaug_autotune_cache_save(str(out).encode()) == OK
    lines = out.read_text().splitlines()
    assert lines[0] == "# ctaug autotune cache v1"
    assert sorted(lines[1:]) == sorted(good.read_text().splitlines()[1:])
    # reloading replaces equal keys instead of duplicating them
    assert L.ctaug_autotune_cache_load(str(out).encode(), None) == OK
    assert L.ctaug_autotune_cache_save(str(out).encode()) == OK
    assert len(out.read_text().splitlines()) == 3
    for bad in ["no header\ngfx950 256 1 4 22 3 16 16 16 0 8176 0\n",
                "# ctaug autotune cache v1\ngfx950 256 1 4 22 3 16 16\n",
                "# ctaug autotune cache v1\ngfx950 256 1 4 22 3 16 16 12 0 8176 0\n",
                "# ctaug autotune cache v1\ngfx950 256 1 4 22 3 16 16 16 0 8176 7\n"]:
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        assert L.ctaug_autotune_cache_load(str(f).encode(), None) == EINVAL
    assert L.ctaug_autotune_cache_load(str(tmp_path / "missing.txt").encode(), None) == EINVAL
    assert L.ctaug_autotune_cache_save(None) == EINVAL
    assert L.ctaug_autotune_cache_clear() == OK
    assert L.ctaug_autotune_cache_save(str(out).encode()) == OK
    assert out.read_text().splitlines() == ["# ctaug autotune cache v1"]


def test_prepared_update_validation(L):
    h = ctypes.c_void_p()
    assert L.ctaug_batch_plan_prepare(None, None, ctypes.byref(h)) == EINVAL
    assert L.ctaug_batch_plan_update_prepared(None, None) == EINVAL
    assert L.ctaug_batch_jobs_destroy(None) == EINVAL


def test_noalloc_backward_validation(L):
    """The allocation-free adjoint validates like the workspace call before
    touching the device."""
    r = ctypes.byref
    img, g = vol((8, 8, 8)), vol((64, 64, 64))
    assert L.ctaug_warp_affine_backward_noalloc(None, mat(), 0.0, None, r(g), None, FAKE,
                                                None) == EINVAL
    assert L.ctaug_warp_affine_backward_noalloc(r(img), mat(), 0.0, None, None, None, FAKE,
                                                None) == EINVAL
    assert L.ctaug_warp_affine_backward_noalloc(r(img), mat(), 0.0, r(photo(flags=1)), r(g),
                                                None, FAKE, None) == EINVAL
    assert L.ctaug_warp_affine_backward_noalloc(r(img), mat(), 0.0, None, r(g),
                                                r(vol((8, 8, 9))), None, None) == ESHAPE
    assert L.ctaug_warp_affine_backward_noalloc(r(img), mat(), 0.0, None,
                                                r(vol((0, 4, 4), data=None)), None, None,
                                                None) == OK


def test_batched_backward_validation(L):
    """The batched adjoint validates every job before anything runs."""
    r = ctypes.byref

    def job(img_dims=(8, 8, 8), dtype=F32, out_dims=(0, 4, 4), gM=None, **ph):
        j = _lib.BwdJob()
        j.img_in = vol(img_dims, dtype)
        j.grad_out = vol(out_dims, data=None if 0 in out_dims else FAKE)
        j.grad_img = _lib.Vol()
        j.grad_M = gM
        j.M = mat()
        j.fill = 0.0
        p = photo(**ph) if ph else photo()
        if not ph:
            p.flags = _lib.CTAUG_PHOTO_NONE
        j.photo = p
        return j

    arr = lambda *js: (_lib.BwdJob * len(js))(*js)
    assert L.ctaug_warp_affine_backward_batch_workspace(0) == 0
    assert L.ctaug_warp_affine_backward_batch_workspace(3) == 3 * 2048 * 12 * 8
    assert L.ctaug_warp_affine_backward_batch(None, 1, None, 0, None) == EINVAL
    assert L.ctaug_warp_affine_backward_batch(arr(job()), 0, None, 0, None) == EINVAL
    # empty outputs, no grad_M: a no-op accepted without a workspace
    assert L.ctaug_warp_affine_backward_batch(arr(job(), job()), 2, None, 0, None) == OK
    assert L.ctaug_warp_affine_backward_batch(arr(job(), job(dtype=I16)), 2, None, 0,
                                              None) == EDTYPE
    assert L.ctaug_warp_affine_backward_batch(arr(job(gM=FAKE)), 1, None, 0, None) == EWORKSPACE
    assert L.ctaug_warp_affine_backward_batch(arr(job(flags=1)), 1, None, 0, None) == EINVAL
    bad = job()
    bad.grad_img = vol((8, 8, 9))
    assert L.ctaug_warp_affine_backward_batch(arr(bad), 1, None, 0, None) == ESHAPE
