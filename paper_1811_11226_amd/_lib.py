"""ctypes declarations of the C ABI in include/ctaug.h (argument marshalling only).

The shared library is loaded lazily from this package directory; if it is
missing, every entry point raises instead of falling back to anything else.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctaug.so")

CTAUG_OK = 0
STATUS_NAMES = {0: "CTAUG_OK", 1: "CTAUG_EINVAL", 2: "CTAUG_EDTYPE", 3: "CTAUG_ESHAPE",
                4: "CTAUG_EWORKSPACE", 5: "CTAUG_EHIP", 6: "CTAUG_ENODEV"}
CTAUG_F32, CTAUG_I16, CTAUG_I8 = 0, 1, 2
CTAUG_PHOTO_WINDOW = 1
CTAUG_PHOTO_OCCLUDE = 2
CTAUG_PHOTO_NONE = 0x80000000


class CtaugError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


class Vol(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dim", ctypes.c_int64 * 3),
                ("stride", ctypes.c_int64 * 3)]


class Photo(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_float), ("offset", ctypes.c_float), ("sigma", ctypes.c_float),
                ("win_lo", ctypes.c_float), ("win_hi", ctypes.c_float), ("gamma", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("volume_id", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("occ_lo", ctypes.c_float), ("occ_hi", ctypes.c_float)]


class AffineParams(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_double * 3), ("scale", ctypes.c_double * 3),
                ("shear", ctypes.c_double * 3), ("reflect", ctypes.c_double * 3),
                ("generic", ctypes.c_double * 9), ("disp", ctypes.c_double * 3),
                ("crop", ctypes.c_double * 3)]


class Job(ctypes.Structure):
    _fields_ = [("img_in", Vol), ("lbl_in", Vol), ("img_out", Vol), ("lbl_out", Vol),
                ("M", ctypes.c_float * 12), ("fill", ctypes.c_float),
                ("label_fill", ctypes.c_int32), ("photo", Photo), ("ctrl", ctypes.c_void_p),
                ("grid", ctypes.c_int64 * 3)]


class BwdJob(ctypes.Structure):
    _fields_ = [("img_in", Vol), ("grad_out", Vol), ("grad_img", Vol),
                ("grad_M", ctypes.c_void_p), ("M", ctypes.c_float * 12), ("fill", ctypes.c_float),
                ("photo", Photo)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32 * 3), ("wg_per_cu", ctypes.c_int32),
                ("lds_cells", ctypes.c_int32), ("lds_format", ctypes.c_int32)]


_P = ctypes.c_void_p
_PV = ctypes.POINTER(Vol)
_PF = ctypes.POINTER(ctypes.c_float)
_PD = ctypes.POINTER(ctypes.c_double)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_S = ctypes.c_int  # ctaug_status

# name -> (restype, argtypes); every symbol declared in include/ctaug.h
SIGNATURES = {
    "ctaug_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ctaug_version": (ctypes.c_int, []),
    "ctaug_affine_matrix": (_S, [ctypes.POINTER(AffineParams), _PI64, _PI64, _PD, _PF]),
    "ctaug_warp_affine": (_S, [_PV, _PV, _PF, ctypes.c_float, ctypes.c_int32,
                               ctypes.POINTER(Photo), _PV, _PV, _P]),
    "ctaug_warp_labels": (_S, [_PV, _PF, ctypes.c_int32, _PV, _P]),
    "ctaug_warp_displacement": (_S, [_PV, _PV, _PF, _P, ctypes.c_float, ctypes.c_int32,
                                     ctypes.POINTER(Photo), _PV, _PV, _P]),
    "ctaug_warp_bspline": (_S, [_PV, _PV, _PF, _P, _PI64, ctypes.c_float, ctypes.c_int32,
                                ctypes.POINTER(Photo), _PV, _PV, _P]),
    "ctaug_photometric_noise": (_S, [_PV, ctypes.POINTER(Photo), _P]),
    "ctaug_noise": (_S, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, _P,
                         _P, _P]),
    "ctaug_box_muller": (_S, [_P, ctypes.c_int64, _P, _P]),
    "ctaug_warp_backward_workspace": (ctypes.c_size_t, [_PI64]),
    "ctaug_warp_affine_backward": (_S, [_PV, _PF, ctypes.c_float, ctypes.POINTER(Photo), _PV,
                                        _PV, _P, _P, ctypes.c_size_t, _P]),
    "ctaug_warp_affine_backward_noalloc": (_S, [_PV, _PF, ctypes.c_float, ctypes.POINTER(Photo),
                                                _PV, _PV, _P, _P]),
    "ctaug_warp_affine_backward_batch_workspace": (ctypes.c_size_t, [ctypes.c_int32]),
    "ctaug_warp_affine_backward_batch": (_S, [ctypes.POINTER(BwdJob), ctypes.c_int32, _P,
                                              ctypes.c_size_t, _P]),
    "ctaug_warp_displacement_backward": (_S, [_PV, _PF, _P, ctypes.c_float, ctypes.POINTER(Photo),
                                              _PV, _PV, _P, _P, _P, ctypes.c_size_t, _P]),
    "ctaug_warp_bspline_backward_workspace": (ctypes.c_size_t, [_PI64, _PI64]),
    "ctaug_warp_bspline_backward": (_S, [_PV, _PF, _P, _PI64, ctypes.c_float,
                                         ctypes.POINTER(Photo), _PV, _PV, _P, _P, _P,
                                         ctypes.c_size_t, _P]),
    "ctaug_bspline_upsample": (_S, [_P, _PI64, _PI64, _P, _P]),
    "ctaug_bspline_adjoint_workspace": (ctypes.c_size_t, [_PI64, _PI64]),
    "ctaug_bspline_upsample_adjoint": (_S, [_P, _PI64, _PI64, _P, _P, ctypes.c_size_t, _P]),
    "ctaug_batch_plan_prepare": (_S, [_P, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_void_p)]),
    "ctaug_batch_plan_update_prepared": (_S, [_P, _P]),
    "ctaug_batch_jobs_destroy": (_S, [_P]),
    "ctaug_autotune_cache_lookup": (_S, [ctypes.POINTER(Job), ctypes.c_int32,
                                         ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_int32)]),
    "ctaug_autotune_cache_save": (_S, [ctypes.c_char_p]),
    "ctaug_autotune_cache_load": (_S, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "ctaug_autotune_cache_clear": (_S, []),
    "ctaug_pipeline_create": (_S, [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "ctaug_pipeline_acquire": (_S, [_P, ctypes.POINTER(ctypes.c_void_p)]),
    "ctaug_pipeline_submit": (_S, [_P, _PV, _PV, _PF, ctypes.c_float, ctypes.c_int32,
                                   ctypes.POINTER(Photo), _PV, _PV]),
    "ctaug_pipeline_stream": (_S, [_P, ctypes.POINTER(ctypes.c_void_p)]),
    "ctaug_pipeline_sync": (_S, [_P]),
    "ctaug_pipeline_destroy": (_S, [_P]),
    "ctaug_batch_plan_create": (_S, [ctypes.POINTER(Job), ctypes.c_int32,
                                     ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_void_p)]),
    "ctaug_batch_plan_update": (_S, [_P, ctypes.POINTER(Job)]),
    "ctaug_batch_plan_launch": (_S, [_P, _P]),
    "ctaug_batch_plan_run": (_S, [_P, _P]),
    "ctaug_batch_plan_capture": (_S, [_P, _P]),
    "ctaug_batch_plan_replay": (_S, [_P, _P]),
    "ctaug_batch_plan_autotune": (_S, [_P, ctypes.POINTER(Tuning), ctypes.c_int32, ctypes.c_int32,
                                       _P, ctypes.POINTER(Tuning), _PF]),
    "ctaug_batch_plan_get_tuning": (_S, [_P, ctypes.POINTER(Tuning)]),
    "ctaug_batch_plan_destroy": (_S, [_P]),
    "ctaug_copy": (_S, [_P, _P, ctypes.c_size_t, _P]),
    "ctaug_resample_sigma": (_S, [_PD, ctypes.c_double, _PF]),
    "ctaug_gaussian_smooth_workspace": (ctypes.c_size_t, [_PI64]),
    "ctaug_gaussian_smooth": (_S, [_PV, _PV, _PF, _P, ctypes.c_size_t, _P]),
}

_lib = None


def load():
    """Load libctaug.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_1811_11226_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, what):
    if status != CTAUG_OK:
        raise CtaugError(status, what)
