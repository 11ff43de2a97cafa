"""MI355X-native TSQR / CAQR (Demmel, Grigori, Hoemmen, Langou, arXiv 0808.2664).

The compute path is libtsqr.so (hand-written HIP kernels for gfx950, C ABI in
include/tsqr.h); this package is the thin Python binding over it.
"""
from .tsqr import BatchPlan, QTree, TSQRFunction, caqr, caqr_left, check_status, cholqr, factor, factor_batched, lstsq, mgs, plan_geometry, qr, qr_backward, sign_normalize, sign_normalize_batched, tsqr  # noqa: F401
from . import _lib  # noqa: F401

__all__ = ["BatchPlan", "QTree", "TSQRFunction", "caqr", "caqr_left", "check_status", "cholqr", "factor", "factor_batched", "lstsq", "mgs", "plan_geometry", "qr", "qr_backward", "sign_normalize", "sign_normalize_batched", "tsqr"]
