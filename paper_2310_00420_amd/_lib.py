"""ctypes declarations of the C ABI in ``include/cmtcs.h`` and the loader of ``libcmtcs.so``.

The shared library is built in-tree by ``paper_2310_00420_amd.build``.  There is no fallback:
if it is missing or fails to load, ``load()`` raises.  ``CMTCS_LIB`` names another build of the
same library to load instead (the host-sanitizer build of the tests).
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CMTCS_LIB") or os.path.join(HERE, "libcmtcs.so")

CMTCS_OK, CMTCS_E_INVALID, CMTCS_E_HIP, CMTCS_E_NOMEM, CMTCS_E_UNSUPPORTED = range(5)
CMTCS_F32, CMTCS_BF16, CMTCS_F16 = range(3)
CMTCS_MATH_F64, CMTCS_MATH_F32, CMTCS_MATH_MIXED = range(3)
CMTCS_OP_DENSE, CMTCS_OP_PARTIAL_FOURIER = range(2)
CMTCS_CG_CONVERGED, CMTCS_CG_MAX_ITER, CMTCS_CG_BREAKDOWN, CMTCS_CG_NONPOS_RITZ = range(4)

STATUS_NAMES = {0: "CMTCS_OK", 1: "CMTCS_E_INVALID", 2: "CMTCS_E_HIP", 3: "CMTCS_E_NOMEM",
                4: "CMTCS_E_UNSUPPORTED"}


class Problem(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("C", ctypes.c_int32), ("D", ctypes.c_int32),
                ("row_off", ctypes.POINTER(ctypes.c_int64)),
                ("phi", ctypes.c_void_p), ("phi_dtype", ctypes.c_int),
                ("phi_resid", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("beta", ctypes.c_double), ("math", ctypes.c_int),
                ("max_rhs", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("max_K", ctypes.c_int32), ("op", ctypes.c_int), ("freq", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("refine_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("em_iter", ctypes.c_uint64), ("probes", ctypes.c_void_p),
                ("alpha_max", ctypes.c_double), ("graph", ctypes.c_int32),
                ("common_probes", ctypes.c_int32), ("precond", ctypes.c_int32)]


class CgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("ritz_min", ctypes.c_void_p), ("ritz_max", ctypes.c_void_p),
                ("k_eff", ctypes.c_void_p)]


_lib = None


def load():
    """Loads libcmtcs.so once and declares its functions."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcmtcs.so is not built (run python -m paper_2310_00420_amd.build): "
                          + LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    vp = ctypes.c_void_p
    lib.cmtcs_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Problem), vp]
    lib.cmtcs_create.restype = st
    lib.cmtcs_destroy.argtypes = [vp]
    lib.cmtcs_destroy.restype = st
    lib.cmtcs_estep.argtypes = [vp, vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp, vp,
                                ctypes.POINTER(CgStats)]
    lib.cmtcs_estep.restype = st
    lib.cmtcs_mstep.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Opts), vp]
    lib.cmtcs_mstep.restype = st
    lib.cmtcs_mstep_pi.argtypes = [vp, vp, vp]
    lib.cmtcs_mstep_pi.restype = st
    lib.cmtcs_log_likelihood.argtypes = [vp, vp, vp, vp, vp]
    lib.cmtcs_log_likelihood.restype = st
    lib.cmtcs_em_iter.argtypes = [vp, vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp, vp]
    lib.cmtcs_em_iter.restype = st
    lib.cmtcs_solve.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp, vp,
                                vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(CgStats)]
    lib.cmtcs_solve.restype = st
    lib.cmtcs_rhs.argtypes = [vp, vp]
    lib.cmtcs_rhs.restype = st
    lib.cmtcs_grad.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp, vp,
                               ctypes.c_double, vp, vp]
    lib.cmtcs_grad.restype = st
    lib.cmtcs_apply.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp, vp]
    lib.cmtcs_apply.restype = st
    lib.cmtcs_apply_noalloc.argtypes = [ctypes.POINTER(Problem), vp, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), vp, vp, vp]
    lib.cmtcs_apply_noalloc.restype = st
    lib.cmtcs_profile.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
    lib.cmtcs_profile.restype = st
    lib.cmtcs_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.cmtcs_tiles.restype = st
    lib.cmtcs_last_error.argtypes = []
    lib.cmtcs_last_error.restype = ctypes.c_char_p
    lib.cmtcs_version.argtypes = []
    lib.cmtcs_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class CmtcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


def check(code):
    if code != CMTCS_OK:
        raise CmtcsError(code, load().cmtcs_last_error().decode())
