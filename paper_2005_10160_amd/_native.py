"""ctypes binding of ``libgravfft.so`` (argument marshalling only).

Every step of the operator runs in the HIP library; this module only
declares the C signatures of ``include/gravfft.h``.  Loading fails loudly
when the library has not been built: there is no other code path.
"""

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgravfft.so")

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EDEVICE, GF_EUNSUPPORTED, GF_EBUSY = range(6)
GF_F64, GF_F32 = 0, 1
GF_OP_FORWARD, GF_OP_ADJOINT = 0, 1

EXPORTED = (
    "gf_plan_create", "gf_plan_create_layered", "gf_plan_create_levels", "gf_plan_destroy", "gf_plan_get_info", "gf_plan_bytes",
    "gf_workspace_bytes", "gf_forward", "gf_adjoint", "gf_status_string",
    "gf_last_error", "gf_debug_kernel_table", "gf_debug_spectrum",
    "gf_plan_set_timing", "gf_plan_last_pass_ms", "gf_debug_fail_alloc", "gf_debug_live_bytes",
    "gf_forward_noalloc", "gf_debug_level_path",
)


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("px", ctypes.c_int), ("py", ctypes.c_int),
        ("n_out", ctypes.c_int), ("n_spec", ctypes.c_int),
        ("components", ctypes.c_uint), ("spec_mask", ctypes.c_uint),
        ("precision", ctypes.c_int), ("max_batch", ctypes.c_int),
        ("spectra_bytes", ctypes.c_size_t), ("internal_workspace_bytes", ctypes.c_size_t),
        ("plan_ms", ctypes.c_double),
        ("n_levels", ctypes.c_int),
        ("col_groups", ctypes.c_int),
        ("level_path", ctypes.c_int),
        ("level_chunk", ctypes.c_int),
    ]


class GravFFTError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (where, status_name(status), detail))


_lock = threading.Lock()
_lib = None


def load(path=None):
    """Load the HIP library (once).  Raises if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise ImportError("libgravfft.so is not built (%s); run `python -m paper_2005_10160_amd.build`" % p)
        lib = ctypes.CDLL(p)
        vp, i, u, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
        pd = ctypes.POINTER(ctypes.c_double)
        lib.gf_plan_create.argtypes = [i, i, i, d, d, d, d, u, i, i, vp, ctypes.POINTER(vp)]
        lib.gf_plan_create.restype = i
        lib.gf_plan_create_layered.argtypes = [i, i, i, d, d, pd, d, u, i, i, vp, ctypes.POINTER(vp)]
        lib.gf_plan_create_layered.restype = i
        lib.gf_plan_create_levels.argtypes = [i, i, i, d, d, d, d, i, u, i, i, vp, ctypes.POINTER(vp)]
        lib.gf_plan_create_levels.restype = i
        lib.gf_plan_destroy.argtypes = [vp]
        lib.gf_plan_destroy.restype = i
        lib.gf_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        lib.gf_plan_get_info.restype = i
        lib.gf_plan_bytes.argtypes = [vp]
        lib.gf_plan_bytes.restype = sz
        lib.gf_workspace_bytes.argtypes = [vp, i, i, ctypes.POINTER(sz)]
        lib.gf_workspace_bytes.restype = i
        lib.gf_forward.argtypes = [vp, vp, vp, i, vp, sz, vp]
        lib.gf_forward.restype = i
        lib.gf_adjoint.argtypes = [vp, vp, vp, i, vp, sz, vp]
        lib.gf_adjoint.restype = i
        lib.gf_status_string.argtypes = [i]
        lib.gf_status_string.restype = ctypes.c_char_p
        lib.gf_last_error.argtypes = []
        lib.gf_last_error.restype = ctypes.c_char_p
        lib.gf_debug_kernel_table.argtypes = [vp, i, pd]
        lib.gf_debug_kernel_table.restype = i
        lib.gf_debug_spectrum.argtypes = [vp, u, i, pd]
        lib.gf_debug_spectrum.restype = i
        lib.gf_plan_set_timing.argtypes = [vp, i]
        lib.gf_plan_set_timing.restype = i
        lib.gf_plan_last_pass_ms.argtypes = [vp, i, pd]
        lib.gf_plan_last_pass_ms.restype = i
        lib.gf_debug_level_path.argtypes = [i, i]
        lib.gf_debug_level_path.restype = i
        lib.gf_forward_noalloc.argtypes = [vp, vp, vp, i, vp]
        lib.gf_forward_noalloc.restype = i
        lib.gf_debug_fail_alloc.argtypes = [i]
        lib.gf_debug_fail_alloc.restype = i
        lib.gf_debug_live_bytes.argtypes = []
        lib.gf_debug_live_bytes.restype = sz
        _lib = lib
        return lib


def status_name(s):
    names = {0: "GF_OK", 1: "GF_EINVAL", 2: "GF_ENOMEM", 3: "GF_EDEVICE", 4: "GF_EUNSUPPORTED", 5: "GF_EBUSY"}
    return names.get(int(s), "GF_UNKNOWN(%d)" % int(s))


def check(status, where):
    if status != GF_OK:
        detail = load().gf_last_error().decode(errors="replace")
        raise GravFFTError(status, where, detail)
