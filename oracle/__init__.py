"""CPU FP64 oracle for the QR path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path
(``paper_0808_2664_amd``) never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C99, FP64, pairwise summation),
built with gcc into ``liboracle.so`` next to this file.  This module only
marshals numpy arrays.  What each function computes and which passage of the
paper it follows is stated in ``oracle.c``; the conventions are:

* Householder vectors with unit topmost entry (paper Sec. 5.2),
  ``beta = -sign(alpha)*||x||``, sign(0) = +1, ``tau = 0`` for a zero tail;
* comparisons are made after the sign normalisation ``D = sign(diag R)``,
  since the factorisation is unique only up to those signs (Sec. 2.1).

``cholqr`` and ``mgs`` are the CholeskyQR and modified Gram-Schmidt the
paper compares TSQR with (Sec. 2.3).  ``geqrf_blocked`` is the same
Householder QR organised in panels with compact-WY trailing updates (the
conventional blocked QR that CAQR reorganises, Sec. 3), multithreaded with
OpenMP, for square matrices too large for the unblocked loop.
``qr_adjoint`` is not from the paper: it is the published QR adjoint
(Walter & Lehmann; Liao et al. "copyltu" form).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (ISO C99, OpenMP, no fast-math, no FMA
    contraction: the vectoriser may not reassociate sums, so every sum keeps
    the order written in the C source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c99", "-O3", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_geqrf.argtypes = [i64, i64, dp, dp]
        lib.oracle_apply_qt.argtypes = [i64, i64, i64, dp, dp, dp]
        lib.oracle_apply_q.argtypes = [i64, i64, i64, dp, dp, dp]
        lib.oracle_form_q.argtypes = [i64, i64, dp, dp, dp]
        lib.oracle_qr_adjoint.argtypes = [i64, i64, dp, dp, dp, dp, dp]
        lib.oracle_lstsq.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_cholqr.argtypes = [i64, i64, dp, dp, dp, ctypes.c_int]
        lib.oracle_geqrf_blocked.argtypes = [i64, i64, dp, dp, i64]
        lib.oracle_mgs.argtypes = [i64, i64, dp, dp, dp]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_psum.argtypes = [dp, i64]
        lib.oracle_psum.restype = ctypes.c_double
        for f in ("oracle_geqrf", "oracle_apply_qt", "oracle_apply_q",
                  "oracle_form_q", "oracle_qr_adjoint", "oracle_lstsq", "oracle_cholqr",
                  "oracle_geqrf_blocked", "oracle_mgs"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(rc: int, name: str):
    if rc != 0:
        raise RuntimeError(f"{name} failed with code {rc}")


def psum(x) -> float:
    x = _f64(x).ravel()
    return float(_load().oracle_psum(_p(x), x.size))


def geqrf(A):
    """Householder QR.  Returns (YR, tau): R in the upper triangle of YR,
    reflector tails below the diagonal (unit top entry implicit)."""
    YR = _f64(A).copy()
    m, n = YR.shape
    tau = np.zeros(n)
    _check(_load().oracle_geqrf(m, n, _p(YR), _p(tau)), "oracle_geqrf")
    return YR, tau


def geqrf_blocked(A, nb: int = 64):
    """Blocked Householder QR (panels of nb columns, compact-WY trailing
    updates, OpenMP over trailing column blocks).  Same outputs as geqrf."""
    YR = _f64(A).copy()
    m, n = YR.shape
    tau = np.zeros(n)
    _check(_load().oracle_geqrf_blocked(m, n, _p(YR), _p(tau), int(nb)), "oracle_geqrf_blocked")
    return YR, tau


def set_threads(nthreads: int = 0) -> int:
    """OpenMP threads of later oracle calls (0: the runtime default);
    returns the count in effect."""
    return int(_load().oracle_set_threads(int(nthreads)))


def apply_qt(YR, tau, B):
    """Q^T B for the full m x m orthogonal Q of geqrf."""
    YR, tau, Bc = _f64(YR), _f64(tau), _f64(B).copy()
    m, n = YR.shape
    vec = Bc.ndim == 1
    if vec:
        Bc = Bc.reshape(m, 1)
    _check(_load().oracle_apply_qt(m, n, Bc.shape[1], _p(YR), _p(tau), _p(Bc)),
           "oracle_apply_qt")
    return Bc.ravel() if vec else Bc


def apply_q(YR, tau, B):
    """Q B for the full m x m orthogonal Q of geqrf."""
    YR, tau, Bc = _f64(YR), _f64(tau), _f64(B).copy()
    m, n = YR.shape
    vec = Bc.ndim == 1
    if vec:
        Bc = Bc.reshape(m, 1)
    _check(_load().oracle_apply_q(m, n, Bc.shape[1], _p(YR), _p(tau), _p(Bc)),
           "oracle_apply_q")
    return Bc.ravel() if vec else Bc


def form_q(YR, tau):
    """Thin Q (m x n) = Q [I_n; 0]."""
    YR, tau = _f64(YR), _f64(tau)
    m, n = YR.shape
    Q = np.empty((m, n))
    _check(_load().oracle_form_q(m, n, _p(YR), _p(tau), _p(Q)), "oracle_form_q")
    return Q


def r_of(YR):
    """Upper triangle (first n rows) of a geqrf result."""
    n = YR.shape[1]
    return np.triu(YR[:n, :])


def signs(R):
    """D = sign(diag R) with sign(0) = +1."""
    d = np.diag(R).copy()
    return np.where(d < 0.0, -1.0, 1.0)


def qr(A):
    """Sign-normalised thin QR (diag(R) >= 0): returns (Q, R)."""
    YR, tau = geqrf(A)
    R = r_of(YR)
    Q = form_q(YR, tau)
    d = signs(R)
    return Q * d[None, :], R * d[:, None]


def qr_adjoint(Q, R, dQ, dR):
    """dA for the sign-normalised thin QR, given upstream dQ, dR."""
    Q, R, dQ, dR = _f64(Q), _f64(R), _f64(dQ), _f64(dR)
    m, n = Q.shape
    dA = np.empty((m, n))
    _check(_load().oracle_qr_adjoint(m, n, _p(Q), _p(R), _p(dQ), _p(dR), _p(dA)),
           "oracle_qr_adjoint")
    return dA


def lstsq(A, B):
    """Least squares min ||A X - B|| column by column (A full column rank):
    returns (X, rnorm), X n x k, rnorm the k residual norms.  A 1-D B gives
    a 1-D X and a scalar rnorm."""
    A, B = _f64(A), _f64(B)
    m, n = A.shape
    vec = B.ndim == 1
    Bc = B.reshape(m, 1) if vec else B
    k = Bc.shape[1]
    X = np.empty((n, k))
    rn = np.empty(k)
    _check(_load().oracle_lstsq(m, n, k, _p(A), _p(np.ascontiguousarray(Bc)), _p(X), _p(rn)),
           "oracle_lstsq")
    return (X.ravel(), float(rn[0])) if vec else (X, rn)


def cholqr(A, passes: int = 1):
    """CholeskyQR (passes = 1) or CholeskyQR2 (passes = 2): returns (Q, R),
    diag(R) > 0.  Raises FloatingPointError if a Cholesky pivot is not
    positive (A^T A not numerically positive definite)."""
    A = _f64(A)
    m, n = A.shape
    Q = np.empty((m, n))
    R = np.empty((n, n))
    rc = _load().oracle_cholqr(m, n, _p(A), _p(Q), _p(R), int(passes))
    if rc == -3:
        raise FloatingPointError("Cholesky pivot not positive")
    _check(rc, "oracle_cholqr")
    return Q, R


def mgs(A):
    """Modified Gram-Schmidt: returns (Q, R), diag(R) > 0.  Raises
    FloatingPointError if a column becomes exactly zero."""
    A = _f64(A)
    m, n = A.shape
    Q = np.empty((m, n))
    R = np.empty((n, n))
    rc = _load().oracle_mgs(m, n, _p(A), _p(Q), _p(R))
    if rc == -3:
        raise FloatingPointError("zero column")
    _check(rc, "oracle_mgs")
    return Q, R


# ---- evaluation helpers (norms of the checks; no factorisation arithmetic) ----

def residual(A, Q, R) -> float:
    """||A - QR||_F / ||A||_F."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - np.asarray(Q, np.float64) @ np.asarray(R, np.float64))
                 / np.linalg.norm(A))


def orthogonality(Q) -> float:
    """||Q^T Q - I||_F."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])))


def rel_err(X, Xref) -> float:
    """Normwise relative error ||X - Xref||_F / ||Xref||_F."""
    Xref = np.asarray(Xref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(X, np.float64) - Xref) / np.linalg.norm(Xref))
