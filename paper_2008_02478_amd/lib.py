"""ctypes binding of libdemag.so: argument types of the C ABI in
include/demag.h, and status checking.  Marshalling only; every step of the
computation runs in the library's HIP kernels."""
import ctypes
import os

LIB_PATH = os.environ.get("DEMAG_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdemag.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4, -5
PBC_X, PBC_Y, PBC_Z = 1, 2, 4
ACCUMULATE = 1
NOALLOC_WORK_BYTES = 64 << 20
TUNE_FORCE = 1
TUNE_KEEP_FORM = 2

_NAMES = {EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", ENOMEM: "ENOMEM", EHIP: "EHIP", ESTATE: "ESTATE"}

_lib = None


class LlgParams(ctypes.Structure):
    """demag_llg_params of include/demag.h."""
    _fields_ = [("Ms", ctypes.c_float), ("A", ctypes.c_float), ("alpha", ctypes.c_float),
                ("gamma", ctypes.c_float), ("dt", ctypes.c_float), ("Hext", ctypes.c_float * 3)]

_vp, _int, _uint, _dbl, _flt = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_float

_SIGS = {
    "demag_setup": [ctypes.POINTER(_vp), _int, _int, _int, _dbl, _dbl, _dbl, _uint, _int],
    "demag_padded_dims": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int)],
    "demag_buffer_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "demag_bind": [_vp, _vp, _vp, _vp],
    "demag_field": [_vp, _vp, _vp, _flt, _vp, _uint, _vp, _vp],
    "demag_field_noalloc": [_vp, _vp, _vp, _flt, _vp, _uint, _vp, _vp],
    "demag_energy": [_vp, _vp, _vp, _flt, _vp, _vp, _vp],
    "demag_backward": [_vp, _vp, _vp, _flt, _vp, _vp, _vp, _uint, _vp],
    "demag_set_timing_events": [_vp, ctypes.POINTER(_vp), _int],
    "demag_setup_batch": [ctypes.POINTER(_vp), _int, ctypes.POINTER(_int), ctypes.POINTER(_dbl),
                          ctypes.POINTER(_dbl), ctypes.POINTER(_int), _uint, _int],
    "demag_batch_layout": [_vp, ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_longlong),
                           ctypes.POINTER(ctypes.c_size_t)],
    "demag_field_batch": [_vp, _vp, _vp, _flt, _vp, _uint, _vp, _vp],
    "demag_backward_batch": [_vp, _vp, _vp, _flt, _vp, _vp, _vp, _uint, _vp],
    "demag_schedule_count": [_vp, ctypes.POINTER(_int)],
    "demag_get_schedule": [_vp, _int, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int)],
    "demag_set_schedule": [_vp, _int, _int, _int, _int],
    "demag_get_z_passes": [_vp, _int, ctypes.POINTER(_int)],
    "demag_set_z_passes": [_vp, _int, _int],
    "demag_autotune": [_vp, _vp, _vp, ctypes.c_char_p, _uint, ctypes.POINTER(_int), _vp],
    "demag_field_2sub": [_vp, _vp, _vp, _flt, _flt, _vp, _uint, _vp, _vp],
    "demag_llg_workspace_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "demag_llg_rk4": [_vp, _vp, ctypes.POINTER(LlgParams), _vp, _vp],
    "demag_setup_oersted": [ctypes.POINTER(_vp), _int, _int, _int, _dbl, _dbl, _dbl, _uint, _int],
    "demag_oersted_field": [_vp, _vp, _flt, _vp, _uint, _vp],
    "demag_stream_copy": [_vp, _vp, ctypes.c_size_t, _vp],
    "demag_destroy": [_vp],
}


class DemagError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load the built library; fails loudly when it is missing (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2008_02478_amd.build_lib`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _int
    lib.demag_last_error.argtypes = []
    lib.demag_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc):
    if rc != OK:
        raise DemagError(rc, load().demag_last_error().decode())
    return rc
