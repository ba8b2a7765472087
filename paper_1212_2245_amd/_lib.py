"""ctypes binding of libdeblur.so: the C ABI of include/deblur.h, argument
marshalling only (every step of the method runs in the library's kernels)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdeblur.so")

DEBLUR_OK = 0
DEBLUR_EINVAL = -1
DEBLUR_EUNSUPPORTED = -2
DEBLUR_EWORKSPACE = -3
DEBLUR_EDEVICE = -4
DEBLUR_ESCRATCH = -5
NOALLOC_SCRATCH_BYTES = 64 << 20

PSF_BOX_H, PSF_BOX_V, PSF_TAPS = 0, 1, 2
BC_REPLICATE, BC_PERIODIC = 0, 1
CONV_AUTO, CONV_RUNSUM, CONV_STENCIL, CONV_FFT = 0, 1, 2, 3
PSI_TV, PSI_PERONA_MALIK = 0, 1
START_FLAT, START_OBSERVED = 0, 1

OP_WIENER, OP_ITERATE, OP_BACKWARD, OP_BACKWARD_WIENER, OP_WIENER_FP64 = 0, 1, 2, 3, 4


class deblur_psf(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("length", ctypes.c_int32), ("ph", ctypes.c_int32),
                ("pw", ctypes.c_int32), ("taps", ctypes.c_void_p), ("frac", ctypes.c_float)]


class deblur_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("eps_data", ctypes.c_float), ("eps_tv", ctypes.c_float),
                ("s_min", ctypes.c_float), ("iters", ctypes.c_int32), ("robust", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("conv", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("psi", ctypes.c_int32), ("rf_lut", ctypes.c_int32), ("bwd_tile", ctypes.c_int32)]


class deblur_batch_item(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("u", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("psf", deblur_psf), ("p", deblur_params), ("K", ctypes.c_double),
                ("pos_floor", ctypes.c_float)]


# (name, restype, argtypes) of every exported entry point
_VP, _SZ, _I32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
_PSF, _PAR = ctypes.POINTER(deblur_psf), ctypes.POINTER(deblur_params)
SIGNATURES = [
    ("deblur_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("deblur_version", ctypes.c_int, []),
    ("deblur_tile_variants", ctypes.c_int, []),
    ("deblur_box_tile_variants", ctypes.c_int, []),
    ("deblur_workspace_bytes", _SZ, [_I32, _I32, _I32, _I32, _PSF, _PAR]),
    ("deblur_wiener", ctypes.c_int, [_VP, _VP, _I32, _I32, _I32, _PSF, ctypes.c_double, ctypes.c_float,
                                     _VP, _SZ, _VP]),
    ("deblur_wiener_fp64", ctypes.c_int, [_VP, _VP, _I32, _I32, _I32, _PSF, ctypes.c_double, ctypes.c_float,
                                          _VP, _SZ, _VP]),
    ("deblur_rrrl_start", ctypes.c_int, [_VP, _VP, _I32, _I32, _I32, _I32, ctypes.c_float, _VP]),
    ("deblur_rrrl_iterate", ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _PSF, _PAR, _VP, _VP, _SZ, _VP]),
    ("deblur_rrrl_iterate_noalloc", ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _PSF, _PAR, _VP, _VP]),
    ("deblur_rrrl_backward", ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _PSF, _PAR, _I32, ctypes.c_double,
                                            ctypes.c_float, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("deblur_workspace_bytes_batch", _SZ, [_I32, _I32, _I32, _I32, _I32, _PSF, _PAR]),
    ("deblur_wiener_batch", ctypes.c_int, [_I32, _VP, _VP, _I32, _I32, _I32, ctypes.c_int64, _PSF, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_float, _I32, _VP, _SZ, _VP]),
    ("deblur_rrrl_iterate_batch", ctypes.c_int, [_I32, _VP, _VP, _VP, _I32, _I32, _I32, ctypes.c_int64, _PSF,
                                                 ctypes.c_int64, _VP, _PAR, _VP, ctypes.c_int64, _VP, _SZ, _VP]),
    ("deblur_rrrl_backward_batch", ctypes.c_int, [_I32, _VP, _VP, _VP, _I32, _I32, _I32, ctypes.c_int64,
                                                  ctypes.c_int64, _PSF, ctypes.c_int64, _VP, _PAR, _I32,
                                                  ctypes.c_double, ctypes.c_float, _VP, _VP, _VP, _VP, _VP, _SZ,
                                                  _VP]),
    ("deblur_batch_plan_create", ctypes.c_int, [ctypes.POINTER(deblur_batch_item), _I32, _I32,
                                                ctypes.POINTER(ctypes.c_void_p)]),
    ("deblur_batch_plan_create_tiled", ctypes.c_int, [ctypes.POINTER(deblur_batch_item), _I32, _I32,
                                                      ctypes.POINTER(_I32), ctypes.POINTER(_VP)]),
    ("deblur_batch_tile_variants", _I32, [_I32]),
    ("deblur_backward_tile_variants", ctypes.c_int, []),
    ("deblur_batch_class_of", _I32, [_VP, _I32]),
    ("deblur_batch_class_tiles", _I32, [_VP, _I32]),
    ("deblur_batch_launch_class", ctypes.c_int, [_VP, _I32, _I32, _VP]),
    ("deblur_batch_run", ctypes.c_int, [_VP, _VP]),
    ("deblur_batch_size", _I32, [_VP]),
    ("deblur_batch_latencies", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double)]),
    ("deblur_batch_plan_destroy", None, [_VP]),
    ("deblur_taps_bytes", _SZ, [_PSF]),
    ("deblur_compile_taps", ctypes.c_int, [_PSF, _VP, _SZ, _VP]),
    ("deblur_rrrl_weights", ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _PSF, _VP, _PAR, _VP]),
    ("deblur_rrrl_update", ctypes.c_int, [_VP, _VP, _VP, _VP, _I32, _I32, _I32, _PSF, _VP, _PAR, _VP]),
]

_lib = None


class DeblurError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        text = load().deblur_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {text} (status {status})")


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m "
                               f"paper_1212_2245_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != DEBLUR_OK:
        raise DeblurError(status, where)
