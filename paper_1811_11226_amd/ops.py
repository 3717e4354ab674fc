"""Python entry points with the names of the C ABI (include/ctaug.h).

Only argument marshalling happens here: torch CUDA tensors provide device
memory and the current HIP stream, and every step runs in the library's
kernels.  Volumes are contiguous [X][Y][Z] tensors (z fastest).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import CTAUG_F32, CTAUG_I16, CTAUG_I8, CTAUG_PHOTO_NONE, CTAUG_PHOTO_WINDOW

_DTYPES = {torch.float32: CTAUG_F32, torch.int16: CTAUG_I16, torch.int8: CTAUG_I8}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require(t, name, dtypes, ndim=3, strided=False):
    """Type/device/rank checks.  strided: t may be a view whose layout the
    library accepts for gathered inputs (z contiguous, x stride a whole number
    of y rows); the library validates the strides themselves."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    if not strided and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def vol(t):
    """ctaug_vol of a tensor: dense volumes pass zero strides, views their
    element strides."""
    v = _lib.Vol()
    v.data = t.data_ptr() if t.numel() > 0 else None
    v.dtype = _DTYPES[t.dtype]
    v.reserved = 0
    for i in range(3):
        v.dim[i] = t.shape[i]
    if t.numel() > 0 and not t.is_contiguous():
        for i in range(3):
            v.stride[i] = t.stride(i)
    return v


def _M32(M):
    a = np.ascontiguousarray(np.asarray(M, dtype=np.float32).reshape(12))
    return (ctypes.c_float * 12)(*a.tolist())


def make_photo(photo):
    """ctypes Photo from any object with gain, offset, sigma, win_lo, win_hi,
    gamma, window, seed and volume_id attributes, and optionally occlude,
    occ_lo and occ_hi (None -> None)."""
    if photo is None:
        return None
    p = _lib.Photo()
    p.gain, p.offset, p.sigma = photo.gain, photo.offset, photo.sigma
    p.win_lo, p.win_hi, p.gamma = photo.win_lo, photo.win_hi, photo.gamma
    p.flags = CTAUG_PHOTO_WINDOW if photo.window else 0
    p.volume_id = int(photo.volume_id)
    p.seed = int(photo.seed)
    if getattr(photo, "occlude", False):
        p.flags |= _lib.CTAUG_PHOTO_OCCLUDE
        p.occ_lo, p.occ_hi = float(photo.occ_lo), float(photo.occ_hi)
    return p


def _ref(x):
    return None if x is None else ctypes.byref(x)


def affine_matrix(prm, in_dim, out_dim):
    """[A|b] from the 27 raw transform draws (FP64 and FP32 copies)."""
    prm = np.asarray(prm, dtype=np.float64).reshape(27)
    p = _lib.AffineParams()
    fields = [("rot", 0, 3), ("scale", 3, 3), ("shear", 6, 3), ("reflect", 9, 3),
              ("generic", 12, 9), ("disp", 21, 3), ("crop", 24, 3)]
    for name, off, n in fields:
        arr = getattr(p, name)
        for i in range(n):
            arr[i] = float(prm[off + i])
    idim = (ctypes.c_int64 * 3)(*[int(v) for v in in_dim])
    odim = (ctypes.c_int64 * 3)(*[int(v) for v in out_dim])
    M64 = (ctypes.c_double * 12)()
    M32 = (ctypes.c_float * 12)()
    _lib.check(_lib.load().ctaug_affine_matrix(ctypes.byref(p), idim, odim, M64, M32),
               "ctaug_affine_matrix")
    return np.array(M64[:], dtype=np.float64), np.array(M32[:], dtype=np.float32)


def _warp(fn_name, img, M, disp, lbl, fill, label_fill, photo, out_dim, out, lbl_out, ctrl=None):
    _require(img, "img", (torch.float32, torch.int16), strided=True)
    if out_dim is None:
        out_dim = tuple(img.shape) if out is None else tuple(out.shape)
    if out is None:
        out = torch.empty(tuple(out_dim), dtype=torch.float32, device=img.device)
    _require(out, "out", (torch.float32,))
    if lbl is not None:
        _require(lbl, "lbl", (torch.int8,), strided=True)
        if lbl_out is None:
            lbl_out = torch.empty(tuple(out.shape), dtype=torch.int8, device=img.device)
        _require(lbl_out, "lbl_out", (torch.int8,))
    vi, vo = vol(img), vol(out)
    vl = vol(lbl) if lbl is not None else None
    vlo = vol(lbl_out) if lbl is not None else None
    ph = make_photo(photo)
    L = _lib.load()
    args = [ctypes.byref(vi), _ref(vl), _M32(M)]
    if disp is not None:
        _require(disp, "disp", (torch.float32,), ndim=4)
        if tuple(disp.shape) != (3,) + tuple(out.shape):
            raise ValueError(f"disp: expected {(3,) + tuple(out.shape)}, got {tuple(disp.shape)}")
        args.append(ctypes.c_void_p(disp.data_ptr() if disp.numel() else None))
    if ctrl is not None:
        _require(ctrl, "ctrl", (torch.float32,), ndim=4)
        if ctrl.shape[0] != 3:
            raise ValueError(f"ctrl: expected [3][Gx][Gy][Gz], got {tuple(ctrl.shape)}")
        args.append(ctypes.c_void_p(ctrl.data_ptr()))
        args.append((ctypes.c_int64 * 3)(*ctrl.shape[1:]))
    st = getattr(L, fn_name)(*args, float(fill), int(label_fill), _ref(ph), ctypes.byref(vo),
                             _ref(vlo), _stream())
    _lib.check(st, fn_name)
    return out, (lbl_out if lbl is not None else None)


def warp_affine(img, M, lbl=None, fill=-1000.0, label_fill=0, photo=None, out_dim=None, out=None,
                lbl_out=None):
    """Fused affine warp + labels + photometrics.  Returns (out, lbl_out)."""
    return _warp("ctaug_warp_affine", img, M, None, lbl, fill, label_fill, photo, out_dim, out,
                 lbl_out)


def warp_labels(lbl, M, out_dim=None, label_fill=0, lbl_out=None):
    """ctaug_warp_labels: nearest-neighbour warp of an int8 label volume alone
    (no image), equal to warp_affine's labels for the same M.  Returns lbl_out."""
    _require(lbl, "lbl", (torch.int8,), strided=True)
    if lbl_out is None:
        shape = tuple(lbl.shape) if out_dim is None else tuple(out_dim)
        lbl_out = torch.empty(shape, dtype=torch.int8, device=lbl.device)
    _require(lbl_out, "lbl_out", (torch.int8,))
    vi, vo = vol(lbl), vol(lbl_out)
    st = _lib.load().ctaug_warp_labels(ctypes.byref(vi), _M32(M), int(label_fill),
                                       ctypes.byref(vo), _stream())
    _lib.check(st, "ctaug_warp_labels")
    return lbl_out


def warp_displacement(img, M, disp, lbl=None, fill=-1000.0, label_fill=0, photo=None,
                      out=None, lbl_out=None):
    """As warp_affine with a dense displacement disp [3][Xo][Yo][Zo] added."""
    out_dim = tuple(disp.shape[1:])
    return _warp("ctaug_warp_displacement", img, M, disp, lbl, fill, label_fill, photo, out_dim,
                 out, lbl_out)


def warp_bspline(img, M, ctrl, lbl=None, fill=-1000.0, label_fill=0, photo=None, out_dim=None,
                 out=None, lbl_out=None):
    """Fused affine + cubic B-spline warp: the displacement of the control grid
    ctrl [3][Gx][Gy][Gz] is evaluated inside the warp kernel (bitwise equal to
    bspline_upsample followed by warp_displacement).  Returns (out, lbl_out)."""
    return _warp("ctaug_warp_bspline", img, M, None, lbl, fill, label_fill, photo, out_dim, out,
                 lbl_out, ctrl=ctrl)


def photometric_noise(volume, photo):
    """In-place photometric chain on a float32 volume."""
    _require(volume, "volume", (torch.float32,))
    v = vol(volume)
    ph = make_photo(photo)
    _lib.check(_lib.load().ctaug_photometric_noise(ctypes.byref(v), ctypes.byref(ph), _stream()),
               "ctaug_photometric_noise")
    return volume


def noise(seed, volume_id, v0, n, gauss=True, words=False, device="cuda"):
    """Gaussians n(v) for v in [v0, v0+n) and/or the Philox words of their groups."""
    g = torch.empty(n, dtype=torch.float32, device=device) if gauss else None
    ng = ((v0 + n - 1) >> 2) - (v0 >> 2) + 1 if n > 0 else 0
    w = torch.empty((ng, 4), dtype=torch.int32, device=device) if words else None
    st = _lib.load().ctaug_noise(int(seed), int(volume_id), int(v0), int(n),
                                 ctypes.c_void_p(g.data_ptr() if g is not None and n else None),
                                 ctypes.c_void_p(w.data_ptr() if w is not None and n else None),
                                 _stream())
    _lib.check(st, "ctaug_noise")
    return g, w   # words as int32 bit patterns [groups][4]


def box_muller(words):
    """Normals from a uint32 word tensor of even length (viewed as int32):
    pairs (radius word, angle word) -> (r cos, r sin)."""
    if words.dtype not in (torch.int32,) or words.numel() % 2 or not words.is_contiguous():
        raise ValueError("box_muller: contiguous int32 tensor of even length expected")
    out = torch.empty(words.numel(), dtype=torch.float32, device=words.device)
    st = _lib.load().ctaug_box_muller(ctypes.c_void_p(words.data_ptr() if words.numel() else None),
                                      words.numel() // 2,
                                      ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                      _stream())
    _lib.check(st, "ctaug_box_muller")
    return out


def warp_backward_workspace(out_dim):
    d = (ctypes.c_int64 * 3)(*[int(v) for v in out_dim])
    return int(_lib.load().ctaug_warp_backward_workspace(d))


def _backward(img, M, grad_out, disp, fill, want_img, want_M, want_disp, photo=None):
    _require(img, "img", (torch.float32, torch.int16), strided=True)
    _require(grad_out, "grad_out", (torch.float32,))
    dev = img.device
    g_img = torch.zeros(tuple(img.shape), dtype=torch.float32, device=dev) if want_img else None
    g_M = torch.empty(12, dtype=torch.float64, device=dev) if want_M else None
    ws_bytes = warp_backward_workspace(grad_out.shape) if want_M else 0
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev) if want_M else None
    vi, vg = vol(img), vol(grad_out)
    vgi = vol(g_img) if want_img else None
    ph = make_photo(photo)
    L = _lib.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else None)
    if disp is None:
        st = L.ctaug_warp_affine_backward(ctypes.byref(vi), _M32(M), float(fill), _ref(ph),
                                          ctypes.byref(vg), _ref(vgi), p(g_M), p(ws), ws_bytes,
                                          _stream())
        _lib.check(st, "ctaug_warp_affine_backward")
        return g_img, g_M
    _require(disp, "disp", (torch.float32,), ndim=4)
    if tuple(disp.shape) != (3,) + tuple(grad_out.shape):
        raise ValueError(f"disp: expected {(3,) + tuple(grad_out.shape)}, got {tuple(disp.shape)}")
    g_disp = torch.empty_like(disp) if want_disp else None
    st = L.ctaug_warp_displacement_backward(ctypes.byref(vi), _M32(M), p(disp), float(fill),
                                            _ref(ph), ctypes.byref(vg), _ref(vgi), p(g_M),
                                            p(g_disp), p(ws), ws_bytes, _stream())
    _lib.check(st, "ctaug_warp_displacement_backward")
    return g_img, g_M, g_disp


def warp_affine_backward(img, M, grad_out, fill=-1000.0, want_img=True, want_M=True,
                         photo=None):
    """(grad_img float32 or None, grad_M float64[12] or None).  photo: the
    forward's photometric parameters without window (gain, offset, noise,
    occlusion), whose adjoint the kernel applies; None = none."""
    return _backward(img, M, grad_out, None, fill, want_img, want_M, False, photo)


def warp_affine_backward_noalloc(img, M, grad_out, fill=-1000.0, photo=None, grad_img=None,
                                 grad_M=None):
    """ctaug_warp_affine_backward_noalloc: the affine adjoint with its scratch
    in the library's static device array.  grad_img (float32, img's dims;
    accumulated into) and grad_M (float64[12]; overwritten) are the caller's
    tensors, either may be None."""
    _require(img, "img", (torch.float32, torch.int16), strided=True)
    _require(grad_out, "grad_out", (torch.float32,))
    vi, vg = vol(img), vol(grad_out)
    vgi = vol(grad_img) if grad_img is not None else None
    ph = make_photo(photo)
    p = ctypes.c_void_p(grad_M.data_ptr()) if grad_M is not None else None
    st = _lib.load().ctaug_warp_affine_backward_noalloc(
        ctypes.byref(vi), _M32(M), float(fill), _ref(ph), ctypes.byref(vg), _ref(vgi), p,
        _stream())
    _lib.check(st, "ctaug_warp_affine_backward_noalloc")
    return grad_img, grad_M


def make_bwd_job(img, M, grad_out, grad_img=None, grad_M=None, fill=-1000.0, photo=None):
    """One job of warp_affine_backward_batch: grad_img (float32, img's dims,
    accumulated into) and grad_M (float64[12], overwritten) are the caller's
    tensors, either may be None."""
    _require(img, "img", (torch.float32, torch.int16), strided=True)
    _require(grad_out, "grad_out", (torch.float32,))
    j = _lib.BwdJob()
    j.img_in = vol(img)
    j.grad_out = vol(grad_out)
    j.grad_img = vol(grad_img) if grad_img is not None else _lib.Vol()
    j.grad_M = grad_M.data_ptr() if grad_M is not None else None
    j.M = _M32(M)
    j.fill = float(fill)
    ph = make_photo(photo)
    if ph is None:
        ph = _lib.Photo()
        ph.flags = CTAUG_PHOTO_NONE
    j.photo = ph
    j._keep = (img, grad_out, grad_img, grad_M)   # the job holds raw device pointers
    return j


def warp_affine_backward_batch(jobs, ws=None):
    """ctaug_warp_affine_backward_batch over a list of make_bwd_job() jobs (or
    a ctypes array of them); ws: a uint8 device tensor of at least
    warp_affine_backward_batch_workspace(len(jobs)) bytes, allocated here
    when None."""
    arr = jobs if isinstance(jobs, ctypes.Array) else (_lib.BwdJob * len(jobs))(*jobs)
    L = _lib.load()
    need = int(L.ctaug_warp_affine_backward_batch_workspace(len(arr)))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    st = L.ctaug_warp_affine_backward_batch(arr, len(arr), ctypes.c_void_p(ws.data_ptr()),
                                            ws.numel(), _stream())
    _lib.check(st, "ctaug_warp_affine_backward_batch")


def warp_affine_backward_batch_workspace(n_jobs):
    return int(_lib.load().ctaug_warp_affine_backward_batch_workspace(int(n_jobs)))


def warp_displacement_backward(img, M, disp, grad_out, fill=-1000.0, want_img=True,
                               want_M=True, want_disp=True, photo=None):
    """(grad_img, grad_M, grad_disp)."""
    return _backward(img, M, grad_out, disp, fill, want_img, want_M, want_disp, photo)


def warp_bspline_backward(img, M, ctrl, grad_out, fill=-1000.0, want_img=True, want_M=True,
                          want_ctrl=True, photo=None):
    """Adjoint of warp_bspline: (grad_img, grad_M float64[12], grad_ctrl
    [3][Gx][Gy][Gz]), each None when not wanted."""
    _require(img, "img", (torch.float32, torch.int16), strided=True)
    _require(grad_out, "grad_out", (torch.float32,))
    _require(ctrl, "ctrl", (torch.float32,), ndim=4)
    if ctrl.shape[0] != 3:
        raise ValueError(f"ctrl: expected [3][Gx][Gy][Gz], got {tuple(ctrl.shape)}")
    dev = img.device
    G = (ctypes.c_int64 * 3)(*ctrl.shape[1:])
    od = (ctypes.c_int64 * 3)(*grad_out.shape)
    L = _lib.load()
    g_img = torch.zeros(tuple(img.shape), dtype=torch.float32, device=dev) if want_img else None
    g_M = torch.empty(12, dtype=torch.float64, device=dev) if want_M else None
    g_ctrl = torch.empty_like(ctrl) if want_ctrl else None
    ws_bytes = int(L.ctaug_warp_bspline_backward_workspace(od, G))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    vi, vg = vol(img), vol(grad_out)
    vgi = vol(g_img) if want_img else None
    ph = make_photo(photo)
    p = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else None)
    st = L.ctaug_warp_bspline_backward(ctypes.byref(vi), _M32(M), p(ctrl), G, float(fill),
                                       _ref(ph), ctypes.byref(vg), _ref(vgi), p(g_M), p(g_ctrl),
                                       p(ws), ws_bytes, _stream())
    _lib.check(st, "ctaug_warp_bspline_backward")
    return g_img, g_M, g_ctrl


def bspline_upsample(ctrl, out_dim, out=None):
    """Dense displacement [3][Xo][Yo][Zo] from a control grid [3][Gx][Gy][Gz]."""
    _require(ctrl, "ctrl", (torch.float32,), ndim=4)
    if out is None:
        out = torch.empty((3,) + tuple(int(v) for v in out_dim), dtype=torch.float32,
                          device=ctrl.device)
    G = (ctypes.c_int64 * 3)(*ctrl.shape[1:])
    od = (ctypes.c_int64 * 3)(*[int(v) for v in out_dim])
    st = _lib.load().ctaug_bspline_upsample(ctypes.c_void_p(ctrl.data_ptr()), G, od,
                                            ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                            _stream())
    _lib.check(st, "ctaug_bspline_upsample")
    return out


def bspline_upsample_adjoint(grad_disp, grid):
    _require(grad_disp, "grad_disp", (torch.float32,), ndim=4)
    G = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    od = (ctypes.c_int64 * 3)(*grad_disp.shape[1:])
    L = _lib.load()
    ws_bytes = int(L.ctaug_bspline_adjoint_workspace(od, G))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=grad_disp.device)
    g = torch.empty((3,) + tuple(int(v) for v in grid), dtype=torch.float32,
                    device=grad_disp.device)
    st = L.ctaug_bspline_upsample_adjoint(
        ctypes.c_void_p(grad_disp.data_ptr() if grad_disp.numel() else None), od, G,
        ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws_bytes, _stream())
    _lib.check(st, "ctaug_bspline_upsample_adjoint")
    return g


def copy(src, dst):
    """Streaming device copy of src into dst (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy: size mismatch")
    _lib.check(_lib.load().ctaug_copy(ctypes.c_void_p(src.data_ptr()),
                                      ctypes.c_void_p(dst.data_ptr()), nbytes, _stream()),
               "ctaug_copy")
    return dst


# ---------------------------------------------------------------------------
# Batch plan
# ---------------------------------------------------------------------------

def make_job(img, M, out, lbl=None, lbl_out=None, fill=-1000.0, label_fill=0, photo=None,
             ctrl=None):
    """One batch job; with ctrl ([3][Gx][Gy][Gz] float32 on the device) the job
    is the B-spline warp of warp_bspline."""
    j = _lib.Job()
    if ctrl is not None:
        _require(ctrl, "ctrl", (torch.float32,), ndim=4)
        j.ctrl = ctrl.data_ptr()
        j.grid = (ctypes.c_int64 * 3)(*ctrl.shape[1:])
    j.img_in = vol(img)
    j.img_out = vol(out)
    if lbl is not None:
        j.lbl_in = vol(lbl)
        j.lbl_out = vol(lbl_out)
    else:
        j.lbl_in = _lib.Vol()
        j.lbl_out = _lib.Vol()
    j.M = _M32(M)
    j.fill = float(fill)
    j.label_fill = int(label_fill)
    ph = make_photo(photo)
    if ph is None:
        ph = _lib.Photo()
        ph.flags = CTAUG_PHOTO_NONE
        ph.gain, ph.gamma, ph.win_hi = 1.0, 1.0, 1.0
    j.photo = ph
    j._keep = (img, out, lbl, lbl_out, ctrl)   # the job holds raw device pointers
    return j


def _job_array(jobs):
    # ctypes copies the structs into the array; the tensors they point to stay
    # referenced from the array
    arr = (_lib.Job * len(jobs))(*jobs)
    arr._keep = [getattr(j, "_keep", None) for j in jobs]
    return arr


class BatchPlan:
    """One persistent launch over a batch of jobs (device job table, pinned
    staging, optional HIP graph, autotuned launch shape)."""

    def __init__(self, jobs, tile=None, wg_per_cu=0, lds_cells=0, lds_format=0):
        self._L = _lib.load()
        arr = jobs if isinstance(jobs, ctypes.Array) else _job_array(jobs)
        tune = None
        if tile is not None:
            tune = _lib.Tuning()
            tune.tile = (ctypes.c_int32 * 3)(*tile)
            tune.wg_per_cu = wg_per_cu
            tune.lds_cells = lds_cells
            tune.lds_format = lds_format
        h = ctypes.c_void_p()
        _lib.check(self._L.ctaug_batch_plan_create(arr, len(jobs), _ref(tune), ctypes.byref(h)),
                   "ctaug_batch_plan_create")
        self._h = h
        self.n = len(jobs)
        self._jobs = arr                # the tensors the device table points to stay alive

    @staticmethod
    def job_array(jobs):
        """The ctypes array of a list of jobs, reusable across update() calls."""
        return _job_array(jobs)

    def update(self, jobs):
        """New job contents: a list of jobs or an array from job_array()."""
        arr = jobs if isinstance(jobs, ctypes.Array) else self.job_array(jobs)
        if len(arr) != self.n:
            raise ValueError(f"expected {self.n} jobs, got {len(arr)}")
        _lib.check(self._L.ctaug_batch_plan_update(self._h, arr), "ctaug_batch_plan_update")
        self._jobs = arr                # the tensors the device table points to stay alive

    def prepare(self, jobs):
        """Descriptors of `jobs` validated and built once, for update_prepared()."""
        arr = jobs if isinstance(jobs, ctypes.Array) else self.job_array(jobs)
        if len(arr) != self.n:
            raise ValueError(f"expected {self.n} jobs, got {len(arr)}")
        return PreparedJobs(self, arr)

    def update_prepared(self, prepared):
        _lib.check(self._L.ctaug_batch_plan_update_prepared(self._h, prepared._h),
                   "ctaug_batch_plan_update_prepared")
        self._jobs = prepared._arr

    def launch(self):
        _lib.check(self._L.ctaug_batch_plan_launch(self._h, _stream()), "ctaug_batch_plan_launch")

    def run(self):
        _lib.check(self._L.ctaug_batch_plan_run(self._h, _stream()), "ctaug_batch_plan_run")

    def capture(self):
        _lib.check(self._L.ctaug_batch_plan_capture(self._h, _stream()), "ctaug_batch_plan_capture")

    def replay(self):
        _lib.check(self._L.ctaug_batch_plan_replay(self._h, _stream()), "ctaug_batch_plan_replay")

    def autotune(self, candidates, reps=5):
        """candidates: (tile, wg_per_cu[, lds_cells[, lds_format]]) tuples."""
        n = len(candidates)
        cand = (_lib.Tuning * n)()
        for i, c in enumerate(candidates):
            cand[i].tile = (ctypes.c_int32 * 3)(*c[0])
            cand[i].wg_per_cu = c[1]
            cand[i].lds_cells = c[2] if len(c) > 2 else 0
            cand[i].lds_format = c[3] if len(c) > 3 else 0
        best = _lib.Tuning()
        times = (ctypes.c_float * n)()
        _lib.check(self._L.ctaug_batch_plan_autotune(self._h, cand, n, reps, _stream(),
                                                     ctypes.byref(best), times),
                   "ctaug_batch_plan_autotune")
        return (tuple(best.tile), best.wg_per_cu, best.lds_cells, best.lds_format), list(times)

    def tuning(self):
        t = _lib.Tuning()
        _lib.check(self._L.ctaug_batch_plan_get_tuning(self._h, ctypes.byref(t)),
                   "ctaug_batch_plan_get_tuning")
        return tuple(t.tile), t.wg_per_cu, t.lds_cells, t.lds_format

    def close(self):
        if getattr(self, "_h", None):
            self._L.ctaug_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedJobs:
    """A batch update prepared for one plan (ctaug_batch_plan_prepare)."""

    def __init__(self, plan, arr):
        self._L = plan._L
        h = ctypes.c_void_p()
        _lib.check(self._L.ctaug_batch_plan_prepare(plan._h, arr, ctypes.byref(h)),
                   "ctaug_batch_plan_prepare")
        self._h = h
        self._arr = arr                 # the jobs' ctypes array stays alive with it

    def close(self):
        if getattr(self, "_h", None):
            self._L.ctaug_batch_jobs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- autotune cache ------------------------------------------------------------

def autotune_cache_lookup(jobs):
    """The cached launch shape (tile, wg_per_cu, lds_cells, lds_format) for a
    batch of jobs on the current device, or None."""
    arr = (_lib.Job * len(jobs))(*jobs)
    t, found = _lib.Tuning(), ctypes.c_int32(0)
    _lib.check(_lib.load().ctaug_autotune_cache_lookup(arr, len(jobs), ctypes.byref(t),
                                                       ctypes.byref(found)),
               "ctaug_autotune_cache_lookup")
    return (tuple(t.tile), t.wg_per_cu, t.lds_cells, t.lds_format) if found.value else None


def autotune_cache_save(path):
    _lib.check(_lib.load().ctaug_autotune_cache_save(str(path).encode()),
               "ctaug_autotune_cache_save")


def autotune_cache_load(path):
    """Merge a saved cache; returns the number of entries read."""
    n = ctypes.c_int32(0)
    _lib.check(_lib.load().ctaug_autotune_cache_load(str(path).encode(), ctypes.byref(n)),
               "ctaug_autotune_cache_load")
    return n.value


def autotune_cache_clear():
    _lib.check(_lib.load().ctaug_autotune_cache_clear(), "ctaug_autotune_cache_clear")


# -- resampling pre-step ------------------------------------------------------

def resample_sigma(spacing, target):
    """Smoothing widths (input voxels) before resampling from voxel spacing
    `spacing` (3 values) to `target`."""
    sp = (ctypes.c_double * 3)(*[float(v) for v in spacing])
    out = (ctypes.c_float * 3)()
    _lib.check(_lib.load().ctaug_resample_sigma(sp, float(target), out), "ctaug_resample_sigma")
    return tuple(out[:])


def gaussian_smooth(volume, sigma, out=None):
    """Separable Gaussian smoothing of a float32 / int16 volume into float32."""
    _require(volume, "volume", (torch.float32, torch.int16))
    if out is None:
        out = torch.empty(tuple(volume.shape), dtype=torch.float32, device=volume.device)
    _require(out, "out", (torch.float32,))
    L = _lib.load()
    d = (ctypes.c_int64 * 3)(*volume.shape)
    ws_bytes = int(L.ctaug_gaussian_smooth_workspace(d))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=volume.device)
    sg = (ctypes.c_float * 3)(*[float(v) for v in sigma])
    vi, vo = vol(volume), vol(out)
    _lib.check(L.ctaug_gaussian_smooth(ctypes.byref(vi), ctypes.byref(vo), sg,
                                       ctypes.c_void_p(ws.data_ptr()), ws_bytes, _stream()),
               "ctaug_gaussian_smooth")
    return out


# ---------------------------------------------------------------------------
# Host-to-device FIFO
# ---------------------------------------------------------------------------

_NP_DTYPES = {np.dtype(np.float32): CTAUG_F32, np.dtype(np.int16): CTAUG_I16,
              np.dtype(np.int8): _lib.CTAUG_I8}


def _host_vol(addr, arr):
    v = _lib.Vol()
    v.data = addr if arr.size else None
    v.dtype = _NP_DTYPES[arr.dtype]
    v.reserved = 0
    for i in range(3):
        v.dim[i] = arr.shape[i]
    return v


class Pipeline:
    """Host-to-device FIFO over `depth` pinned slots of `slot_bytes` bytes:
    put() copies a host volume (and labels) into the next pinned slot (the
    producer's work), then queues its transfer and its fused affine warp; the
    transfer of one volume overlaps the warps of earlier ones."""

    def __init__(self, depth, slot_bytes):
        h = ctypes.c_void_p()
        _lib.check(_lib.load().ctaug_pipeline_create(int(depth), int(slot_bytes), ctypes.byref(h)),
                   "ctaug_pipeline_create")
        self._h = h
        self.slot_bytes = int(slot_bytes)

    @staticmethod
    def slot_bytes_for(img_shape, img_dtype=np.int16, labels=True):
        n = int(np.prod(img_shape))
        b = (n * np.dtype(img_dtype).itemsize + 255) // 256 * 256
        return b + (n if labels else 0)

    def acquire(self):
        """Address of the next pinned host slot (blocks until it is free)."""
        slot = ctypes.c_void_p()
        _lib.check(_lib.load().ctaug_pipeline_acquire(self._h, ctypes.byref(slot)),
                   "ctaug_pipeline_acquire")
        return slot.value

    def submit(self, img_addr, img_like, M, lbl_addr=None, lbl_like=None, fill=-1000.0,
               label_fill=0, photo=None, out=None, lbl_out=None):
        """Queue the acquired slot; img_like / lbl_like give dtype and shape of the
        volumes at host addresses img_addr / lbl_addr inside the slot."""
        vi = _host_vol(img_addr, img_like)
        vl = _host_vol(lbl_addr, lbl_like) if lbl_like is not None else None
        _require(out, "out", (torch.float32,))
        vo = vol(out)
        vlo = vol(lbl_out) if lbl_out is not None else None
        st = _lib.load().ctaug_pipeline_submit(self._h, ctypes.byref(vi), _ref(vl), _M32(M),
                                               float(fill), int(label_fill),
                                               _ref(make_photo(photo)), ctypes.byref(vo),
                                               _ref(vlo))
        _lib.check(st, "ctaug_pipeline_submit")

    def put(self, img, M, lbl=None, fill=-1000.0, label_fill=0, photo=None, out=None,
            lbl_out=None):
        """Copy numpy volumes into the next slot and queue them."""
        img = np.ascontiguousarray(img)
        off = (img.nbytes + 255) // 256 * 256
        need = off + (lbl.nbytes if lbl is not None else 0)
        if need > self.slot_bytes:
            raise ValueError(f"volume needs {need} bytes, slots hold {self.slot_bytes}")
        addr = self.acquire()
        ctypes.memmove(addr, img.ctypes.data, img.nbytes)
        lbl_addr = None
        if lbl is not None:
            lbl = np.ascontiguousarray(lbl)
            lbl_addr = addr + off
            ctypes.memmove(lbl_addr, lbl.ctypes.data, lbl.nbytes)
        self.submit(addr, img, M, lbl_addr, lbl, fill, label_fill, photo, out, lbl_out)

    def stream(self):
        s = ctypes.c_void_p()
        _lib.check(_lib.load().ctaug_pipeline_stream(self._h, ctypes.byref(s)),
                   "ctaug_pipeline_stream")
        return s.value

    def sync(self):
        _lib.check(_lib.load().ctaug_pipeline_sync(self._h), "ctaug_pipeline_sync")

    def close(self):
        if self._h is not None and self._h.value:
            _lib.check(_lib.load().ctaug_pipeline_destroy(self._h), "ctaug_pipeline_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
