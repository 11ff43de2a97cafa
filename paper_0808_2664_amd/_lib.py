"""ctypes binding of libtsqr.so (argument marshalling only).

Every entry point of ``include/tsqr.h`` has a same-named attribute here.  The
library is loaded from this package directory; if it is missing the import
fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsqr.so")

TSQR_F32 = 0
TSQR_F64 = 1
TSQR_SUCCESS = 0
TSQR_ERR_HIP = 1
TSQR_ERR_NOMEM = 2
TSQR_ERR_PLAN = 3
TSQR_ERR_UNSUPPORTED = 4
TSQR_ERR_TIMEOUT = 5
TSQR_ERR_SCRATCH = 6
TSQR_MAX_N = 64
TSQR_FLAG_TREE_LEVELWISE = 1
TSQR_FLAG_ONE_WAVE = 2
TSQR_FLAG_SHARED_CUS = 4


class TsqrOpts(ctypes.Structure):
    _fields_ = [("block_rows", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("arity", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("max_polls", ctypes.c_int32)]


class TsqrError(RuntimeError):
    def __init__(self, func: str, code: int, hip: int = 0):
        self.code = code
        self.hip = hip
        msg = "%s returned %d (%s)" % (func, code, _status(code))
        if hip:
            msg += ", last HIP error %d" % hip
        super().__init__(msg)


_lib = None


def _status(code: int) -> str:
    try:
        return load().tsqr_status_string(code).decode()
    except Exception:  # pragma: no cover
        return "?"


def load():
    """Load libtsqr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtsqr.so not built: run `python -m paper_0808_2664_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    p64 = ctypes.POINTER(ctypes.c_int64)
    popts = ctypes.POINTER(TsqrOpts)
    sig = {
        "tsqr_factor": [i32, i64, i64, vp, i64, vp, i64, popts, ctypes.POINTER(vp), vp],
        "tsqr_apply_qt": [vp, i64, vp, i64, vp],
        "tsqr_apply_q": [vp, i64, vp, i64, vp],
        "tsqr_lstsq": [i32, i64, i64, vp, i64, i64, vp, i64, vp, popts, vp],
        "tsqr_cholqr": [i32, i64, i64, vp, i64, vp, i64, vp, i64, i32, vp],
        "tsqr_mgs": [i32, i64, i64, vp, i64, vp, i64, vp, i64, vp],
        "tsqr_form_q": [vp, vp, i64, vp],
        "tsqr_qtree_destroy": [vp],
        "tsqr_qtree_info": [vp, p64],
        "tsqr_plan_geometry": [i64, i64, popts, p64],
        "tsqr_sign_normalize": [i32, i64, i64, vp, i64, vp, i64, vp],
        "tsqr_last_hip_error": [],
        "tsqr_check_status": [vp],
        "tsqr_apply_layout": [vp, i64, i64],
        "tsqr_factor_batched": [i32, i64, i64, i64, vp, i64, vp, i64, i64, popts, ctypes.POINTER(vp), vp],
        "tsqr_qtree_members": [vp, p64],
        "tsqr_sign_normalize_batched": [i32, i64, i64, i64, vp, i64, vp, i64, i64, vp],
        "tsqr_factor_noalloc": [i32, i64, i64, vp, i64, vp, i64, popts, vp],
        "tsqr_set_phase_events": [i32, vp, vp],
        "caqr_factor": [i32, i64, i64, vp, i64, i64, i32, popts, ctypes.POINTER(vp), vp],
        "tsqr_release_workspace_pools": [],
        "tsqr_form_q_signed": [vp, vp, i64, vp, i64, i64, vp],
        "caqr_factor_left": [i32, i64, i64, vp, i64, i64, i64, i32, popts, ctypes.POINTER(vp), vp],
        "tsqr_copy_r": [i32, i64, vp, i64, vp, i64, vp],
        "tsqr_backward": [i32, i64, i64, i64, vp, i64, i64, vp, i64, i64, vp, i64, i64, vp, i64, i64,
                          vp, i64, i64, vp],
        "tsqr_batch_plan_create": [i32, ctypes.c_int32, p64, p64, popts, ctypes.POINTER(vp)],
        "tsqr_batch_factor": [vp, vp, vp, vp, vp, vp],
        "tsqr_batch_plan_info": [vp, p64],
        "tsqr_batch_plan_destroy": [vp],
        "tsqr_release_streams": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.tsqr_factor_noalloc_scratch_bytes.argtypes = []
    lib.tsqr_factor_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.tsqr_status_string.argtypes = [ctypes.c_int]
    lib.tsqr_status_string.restype = ctypes.c_char_p
    _lib = lib
    atexit.register(_release_at_exit)
    return lib


def _release_at_exit():
    # no library-held CU-masked stream left when the process ends
    if _lib is not None:
        try:
            _lib.tsqr_release_streams()
            _lib.tsqr_release_workspace_pools()
        except Exception:
            pass


def check(func: str, code: int):
    if code != 0:
        raise TsqrError(func, code, load().tsqr_last_hip_error())


def opts(block_rows: int = 0, chains: int = 0, arity: int = 0, flags: int = 0, max_polls: int = 0):
    return TsqrOpts(block_rows, chains, arity, flags, max_polls)
