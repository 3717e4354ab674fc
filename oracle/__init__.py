"""ctypes shim over the plain-C CPU oracle (ctaug_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never imports it.

All arrays are C-contiguous NumPy arrays in [X][Y][Z] order (z fastest).
Floating-point results are float64; parity-mode coordinates are FP32-pinned.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctaug_oracle.c")
_LIB = os.path.join(_HERE, "libctaug_oracle.so")
_lib = None

_CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared"]


def build():
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    cmd = ["gcc", *_CFLAGS, "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_dbl = ctypes.c_double


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_p, _p, _p]
    L.orc_philox4x32_10.restype = None
    L.orc_noise_words.argtypes = [_u64, _u32, _u64, _i64, _p]
    L.orc_noise_words.restype = None
    L.orc_uniform.argtypes = [_u32]
    L.orc_uniform.restype = _dbl
    L.orc_gauss.argtypes = [_u64, _u32, _u64]
    L.orc_gauss.restype = _dbl
    L.orc_box_muller.argtypes = [_p, _i64, _p]
    L.orc_box_muller.restype = None
    L.orc_gauss_range.argtypes = [_u64, _u32, _u64, _i64, _p]
    L.orc_gauss_range.restype = None
    L.orc_photometric.argtypes = [_p, _i64, _p, _int, _u64, _u32, _p, _i64, _p]
    L.orc_photometric.restype = _int
    L.orc_photometric_adjoint.argtypes = [_p, _i64, _p, _int, _p, _i64, _p]
    L.orc_photometric_adjoint.restype = _int
    L.orc_affine_matrix.argtypes = [_p, _p, _p, _p]
    L.orc_affine_matrix.restype = _int
    L.orc_warp.argtypes = [_p, _p, _p, _p, _p, _int, _p, _dbl, _int, _p, _int, _u64, _u32, _p,
                           _p, _p, _p]
    L.orc_warp.restype = _int
    L.orc_warp_points.argtypes = [_p, _p, _p, _p, _p, _int, _p, _dbl, _int, _p, _int, _u64, _u32,
                                  _p, _p, _p, _i64, _p, _p]
    L.orc_warp_points.restype = _int
    L.orc_warp_backward.argtypes = [_p, _p, _p, _p, _int, _p, _dbl, _p, _p, _p, _p, _p]
    L.orc_warp_backward.restype = _int
    L.orc_bspline_upsample.argtypes = [_p, _p, _p, _p]
    L.orc_bspline_upsample.restype = _int
    L.orc_bspline_upsample_f32.argtypes = [_p, _p, _p, _p]
    L.orc_bspline_upsample_f32.restype = _int
    L.orc_bspline_adjoint.argtypes = [_p, _p, _p, _p]
    L.orc_bspline_adjoint.restype = _int
    L.orc_resample_sigma.argtypes = [_p, _dbl, _p]
    L.orc_resample_sigma.restype = None
    L.orc_gaussian_smooth.argtypes = [_p, _p, _p, _p]
    L.orc_gaussian_smooth.restype = _int


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _dims(d):
    return np.asarray(d, dtype=np.int64)


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle returned error {rc}")


# -- noise ----------------------------------------------------------------

def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def noise_words(seed, vol, group0, ngroups):
    out = np.zeros((ngroups, 4), dtype=np.uint32)
    lib().orc_noise_words(seed, vol, group0, ngroups, _ptr(out))
    return out


def uniform(w):
    return lib().orc_uniform(int(w))


def gauss(seed, vol, v0, n):
    out = np.zeros(n, dtype=np.float64)
    lib().orc_gauss_range(seed, vol, v0, n, _ptr(out))
    return out


def box_muller(words):
    w = np.ascontiguousarray(words, dtype=np.uint32).ravel()
    out = np.empty(w.size, dtype=np.float64)
    lib().orc_box_muller(_ptr(w), w.size // 2, _ptr(out))
    return out


def _photo6(photo):
    return np.asarray(photo.as_tuple6(), dtype=np.float64)


def _occ(photo):
    pair = photo.occ_pair() if photo is not None else None
    return None if pair is None else np.asarray(pair, dtype=np.float64)


def photometric(vin, photo):
    """Apply the occlusion and photometric chain of `photo` (a
    synth.PhotoParams) to the FP64 array `vin` ([X][Y][Z] or flat), voxel
    index = position in the array, z = index mod the last axis."""
    v = _c(vin, np.float64).ravel()
    out = np.empty_like(v)
    ph = _photo6(photo)
    occ = _occ(photo)
    Z = int(np.shape(vin)[-1]) if np.ndim(vin) else 1
    _check(lib().orc_photometric(_ptr(v), v.size, _ptr(ph), int(bool(photo.window)),
                                 int(photo.seed), int(photo.volume_id), _ptr(occ), Z, _ptr(out)))
    return out.reshape(np.shape(vin))


def photometric_adjoint(g, photo):
    """Adjoint of the photometric chain without window: gain * g off the
    occluded slab, 0 on it (z = index mod the last axis)."""
    gv = _c(g, np.float64).ravel()
    out = np.empty_like(gv)
    ph = _photo6(photo)
    occ = _occ(photo)
    Z = int(np.shape(g)[-1]) if np.ndim(g) else 1
    _check(lib().orc_photometric_adjoint(_ptr(gv), gv.size, _ptr(ph), int(bool(photo.window)),
                                         _ptr(occ), Z, _ptr(out)))
    return out.reshape(np.shape(g))


# -- transform ------------------------------------------------------------

def affine_matrix(prm, in_dim, out_dim):
    p = _c(prm, np.float64)
    idim, odim = _dims(in_dim), _dims(out_dim)   # keep the arrays alive across the call
    M = np.zeros(12, dtype=np.float64)
    _check(lib().orc_affine_matrix(_ptr(p), _ptr(idim), _ptr(odim), _ptr(M)))
    return M


# -- warp -----------------------------------------------------------------

def warp(img, M, out_dim, lbl=None, disp=None, fill=-1000.0, label_fill=0, photo=None,
         exact=False, want_img=True, want_lbl=None):
    """Forward warp.  M: 12 values [A|b] row-major; FP32-pinned unless
    exact=True (then used in FP64).  Returns (out float64 or None, labels
    int8 or None)."""
    img64 = _c(img, np.float64)
    in_dim = _dims(img64.shape)
    od = _dims(out_dim)
    if want_lbl is None:
        want_lbl = lbl is not None
    lbl8 = _c(lbl, np.int8)
    Mf = np.asarray(M, dtype=np.float32)
    Md = np.asarray(M, dtype=np.float64)
    d = _c(disp, np.float32)
    out = np.empty(tuple(od), dtype=np.float64) if want_img else None
    lout = np.empty(tuple(od), dtype=np.int8) if want_lbl else None
    ph = _photo6(photo) if photo is not None else None
    seed = int(photo.seed) if photo is not None else 0
    vol = int(photo.volume_id) if photo is not None else 0
    window = int(bool(photo.window)) if photo is not None else 0
    occ = _occ(photo)
    _check(lib().orc_warp(_ptr(img64), _ptr(in_dim), _ptr(lbl8), _ptr(Mf), _ptr(Md), int(exact),
                          _ptr(d), float(fill), int(label_fill), _ptr(ph), window, seed, vol,
                          _ptr(occ), _ptr(od), _ptr(out), _ptr(lout)))
    return out, lout


def warp_points(img, M, out_dim, idx, lbl=None, disp=None, fill=-1000.0, label_fill=0,
                photo=None, exact=False, want_img=True, want_lbl=None):
    """The forward warp at the output voxels with linear indices idx only
    (same arithmetic as warp).  Returns (values float64 [len(idx)] or None,
    labels int8 [len(idx)] or None)."""
    img64 = _c(img, np.float64)
    in_dim = _dims(img64.shape)
    od = _dims(out_dim)
    if want_lbl is None:
        want_lbl = lbl is not None
    ix = _c(idx, np.int64).ravel()
    lbl8 = _c(lbl, np.int8)
    Mf = np.asarray(M, dtype=np.float32)
    Md = np.asarray(M, dtype=np.float64)
    d = _c(disp, np.float32)
    out = np.empty(ix.size, dtype=np.float64) if want_img else None
    lout = np.empty(ix.size, dtype=np.int8) if want_lbl else None
    ph = _photo6(photo) if photo is not None else None
    seed = int(photo.seed) if photo is not None else 0
    vol = int(photo.volume_id) if photo is not None else 0
    window = int(bool(photo.window)) if photo is not None else 0
    occ = _occ(photo)
    _check(lib().orc_warp_points(_ptr(img64), _ptr(in_dim), _ptr(lbl8), _ptr(Mf), _ptr(Md),
                                 int(exact), _ptr(d), float(fill), int(label_fill), _ptr(ph),
                                 window, seed, vol, _ptr(occ), _ptr(od), _ptr(ix), ix.size,
                                 _ptr(out), _ptr(lout)))
    return out, lout


def warp_backward(img, M, g, disp=None, fill=-1000.0, exact=False, want_img=True, want_M=True,
                  want_u=False, photo=None):
    """Adjoint of the warp (after the adjoint of the photometric chain
    `photo`, without window, when given).  Returns (g_img float64 [in dims]
    or None, g_M float64 [12] or None, g_u float64 [3][out dims] or None)."""
    img64 = _c(img, np.float64)
    in_dim = _dims(img64.shape)
    g64 = _c(g, np.float64) if photo is None else photometric_adjoint(g, photo)
    od = _dims(g64.shape)
    Mf = np.asarray(M, dtype=np.float32)
    Md = np.asarray(M, dtype=np.float64)
    d = _c(disp, np.float32)
    g_img = np.zeros(img64.shape, dtype=np.float64) if want_img else None
    g_M = np.zeros(12, dtype=np.float64) if want_M else None
    g_u = np.zeros((3,) + tuple(od), dtype=np.float64) if want_u else None
    _check(lib().orc_warp_backward(_ptr(img64), _ptr(in_dim), _ptr(Mf), _ptr(Md), int(exact),
                                   _ptr(d), float(fill), _ptr(g64), _ptr(od), _ptr(g_img),
                                   _ptr(g_M), _ptr(g_u)))
    return g_img, g_M, g_u


# -- B-spline displacement --------------------------------------------------

def bspline_upsample(ctrl, out_dim):
    c = _c(ctrl, np.float64)
    G = _dims(c.shape[1:])
    od = _dims(out_dim)
    u = np.empty((3,) + tuple(od), dtype=np.float64)
    _check(lib().orc_bspline_upsample(_ptr(c), _ptr(G), _ptr(od), _ptr(u)))
    return u


def bspline_upsample_f32(ctrl, out_dim):
    """Parity-mode field (float32, roundings fixed as the fused warp's)."""
    c = _c(ctrl, np.float32)
    G = _dims(c.shape[1:])
    od = _dims(out_dim)
    u = np.empty((3,) + tuple(int(v) for v in out_dim), dtype=np.float32)
    _check(lib().orc_bspline_upsample_f32(_ptr(c), _ptr(G), _ptr(od), _ptr(u)))
    return u


def bspline_adjoint(g_u, grid):
    g = _c(g_u, np.float64)
    od = _dims(g.shape[1:])
    G = _dims(grid)
    out = np.empty((3,) + tuple(G), dtype=np.float64)
    _check(lib().orc_bspline_adjoint(_ptr(g), _ptr(od), _ptr(G), _ptr(out)))
    return out


# -- resampling pre-step ----------------------------------------------------

def resample_sigma(spacing, target):
    """Smoothing sigma per axis (input voxels) before resampling a volume of
    voxel spacing `spacing` to `target`."""
    sp = _c(spacing, np.float64)
    out = np.zeros(3, dtype=np.float64)
    lib().orc_resample_sigma(_ptr(sp), float(target), _ptr(out))
    return out


def gaussian_smooth(img, sigma):
    """Separable Gaussian smoothing (FP64) of a [X][Y][Z] volume."""
    v = _c(img, np.float64)
    d = _dims(v.shape)
    sg = _c(sigma, np.float64)
    out = np.empty_like(v)
    _check(lib().orc_gaussian_smooth(_ptr(v), _ptr(d), _ptr(sg), _ptr(out)))
    return out
