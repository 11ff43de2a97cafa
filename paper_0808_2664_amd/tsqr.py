"""Python API over the C ABI (torch tensors for device memory and streams).

All arithmetic runs in the HIP kernels of libtsqr.so; this module only passes
pointers, sizes and the current HIP stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.TSQR_F64
    if t.dtype == torch.float32:
        return _lib.TSQR_F32
    raise TypeError("only float32 and float64 are supported, got %s" % t.dtype)


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if not t.is_cuda:
        raise ValueError("expected a device (cuda/hip) tensor")
    if t.stride(1) != 1 and t.size(1) > 1:
        raise ValueError("expected a row-major tensor (unit column stride)")
    return max(t.stride(0), t.size(1), 1)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _opts(block_rows=0, chains=0, arity=0, flags=0, max_polls=0):
    if not (block_rows or chains or arity or flags or max_polls):
        return None
    o = _lib.opts(block_rows, chains, arity, flags, max_polls)
    return ctypes.byref(o)


def check_status(stream=None) -> int:
    """Wait for `stream` (default: the current stream) and return the
    library's status for the current device: 0, or TSQR_ERR_TIMEOUT if a
    bounded wait inside a factorisation gave up since the last check."""
    lib = _lib.load()
    st = torch.cuda.current_stream() if stream is None else stream
    rc = lib.tsqr_check_status(ctypes.c_void_p(st.cuda_stream))
    if rc not in (0, _lib.TSQR_ERR_TIMEOUT):
        _lib.check("tsqr_check_status", rc)
    return rc


def plan_geometry(m: int, n: int, block_rows=0, chains=0, arity=0) -> dict:
    """Tree geometry for an m x n TSQR (host only, no GPU work)."""
    lib = _lib.load()
    out = (ctypes.c_int64 * 7)()
    _lib.check("tsqr_plan_geometry", lib.tsqr_plan_geometry(m, n, _opts(block_rows, chains, arity), out))
    keys = ("block_rows", "chain_rows", "chains", "arity", "levels", "blocks", "padded_n")
    return dict(zip(keys, (int(v) for v in out)))


class QTree:
    """Implicit Q of a TSQR (or CAQR) factorisation: the tree of Q factors."""

    def __init__(self, handle: ctypes.c_void_p, A: torch.Tensor, m: int, n: int):
        self._h = handle
        self._A = A  # the reflectors live in A's storage
        self.m = m
        self.n = n
        self.dtype = A.dtype
        self.device = A.device

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = (ctypes.c_int64 * 10)()
        _lib.check("tsqr_qtree_info", _lib.load().tsqr_qtree_info(self._h, out))
        keys = ("m", "n", "block_rows", "chains", "arity", "levels", "blocks", "dtype", "kind", "panel")
        return dict(zip(keys, (int(v) for v in out)))

    def wide_layout(self, k: int, panel: int = 0) -> bool:
        """Whether applies with k columns take the wide kernels (panel: the
        CAQR panel whose tree is applied; 0 for TSQR)."""
        rc = _lib.load().tsqr_apply_layout(self._h, panel, k)
        if rc < 0:
            _lib.check("tsqr_apply_layout", rc)
        return rc == 1

    def _check_b(self, B: torch.Tensor):
        if B.dtype != self.dtype or B.device != self.device:
            raise ValueError("B must match the factor's dtype and device")
        if B.dim() != 2 or B.size(0) != self.m:
            raise ValueError("B must be %d x k" % self.m)

    def apply_qt(self, B: torch.Tensor) -> torch.Tensor:
        """B <- Q^T B in place (full m x m Q)."""
        self._check_b(B)
        _lib.check("tsqr_apply_qt",
                   _lib.load().tsqr_apply_qt(self._h, B.size(1), _ptr(B), _ld(B), _stream(B)))
        return B

    def apply_q(self, B: torch.Tensor) -> torch.Tensor:
        """B <- Q B in place (full m x m Q)."""
        self._check_b(B)
        _lib.check("tsqr_apply_q",
                   _lib.load().tsqr_apply_q(self._h, B.size(1), _ptr(B), _ld(B), _stream(B)))
        return B

    def form_q(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """Explicit thin Q (m x n)."""
        Q = out if out is not None else torch.empty(self.m, self.n, dtype=self.dtype, device=self.device)
        _lib.check("tsqr_form_q", _lib.load().tsqr_form_q(self._h, _ptr(Q), _ld(Q), _stream(Q)))
        return Q

    def form_q_signed(self, R: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Explicit thin Q with the signs of diag(R) folded in: Q <- Q D and
        R <- D R (in place), D = diag(sign R_jj), in the explicit-Q pass
        itself.  R: n x n, or members x n x n for a batched factorisation."""
        Q = out if out is not None else torch.empty(self.m, self.n, dtype=self.dtype, device=self.device)
        if R.dtype != self.dtype or R.device != self.device or R.size(-1) != self.n or R.stride(-1) != 1:
            raise ValueError("R must be the factor's n x n R (or a batch of them)")
        sr = R.stride(0) if R.dim() == 3 else 0
        _lib.check("tsqr_form_q_signed", _lib.load().tsqr_form_q_signed(
            self._h, _ptr(Q), _ld(Q), _ptr(R), R.stride(-2), sr, _stream(Q)))
        return Q

    def close(self):
        if self._h is not None:
            _lib.load().tsqr_qtree_destroy(self._h)
            self._h = None
            self._A = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor(A: torch.Tensor, R: torch.Tensor | None = None, block_rows=0, chains=0, arity=0,
           levelwise: bool = False, want_q: bool = True, max_polls: int = 0, one_wave: bool = False):
    """TSQR of A (m x n, m >= n, n <= 64), IN PLACE: A is overwritten by the
    leaf reflectors.  Returns (R, QTree); diag(R) carries the Householder
    signs (see sign_normalize).  levelwise: reduce the tree node by node
    (TSQR_FLAG_TREE_LEVELWISE) instead of panel-pipelined; same result.
    want_q=False: R only (no implicit Q is formed); returns (R, None).
    max_polls: bound of the pipelined tree's waits (tsqr_opts.max_polls;
    0 = the library default), for tests of the give-up path.  one_wave:
    TSQR_FLAG_ONE_WAVE (the one-wave chain engine everywhere; same bits)."""
    lib = _lib.load()
    m, n = A.shape
    if R is None:
        R = torch.empty(n, n, dtype=A.dtype, device=A.device)
    h = ctypes.c_void_p()
    flags = (_lib.TSQR_FLAG_TREE_LEVELWISE if levelwise else 0) | (_lib.TSQR_FLAG_ONE_WAVE if one_wave else 0)
    rc = lib.tsqr_factor(_dtype_code(A), m, n, _ptr(A), _ld(A), _ptr(R), _ld(R),
                         _opts(block_rows, chains, arity, flags, max_polls), ctypes.byref(h) if want_q else None,
                         _stream(A))
    _lib.check("tsqr_factor", rc)
    return R, (QTree(h, A, m, n) if want_q else None)


def factor_batched(A: torch.Tensor, R: torch.Tensor | None = None, chains=0, arity=0, levelwise: bool = False,
                   want_q: bool = True):
    """TSQR of every matrix of a contiguous [batch, m, n] tensor (n <= 64),
    IN PLACE: A is overwritten by the leaf reflectors.  Each member has its
    own tree (chains = chains per member, a power of the arity; 0 = the
    library's choice).  Returns (R [batch, n, n], QTree over the stacked
    (batch*m) x n rows) or (R, None) without an implicit Q."""
    lib = _lib.load()
    if A.dim() != 3 or not A.is_contiguous():
        raise ValueError("expected a contiguous [batch, m, n] tensor")
    b, m, n = A.shape
    if R is None:
        R = torch.empty(b, n, n, dtype=A.dtype, device=A.device)
    h = ctypes.c_void_p()
    flags = _lib.TSQR_FLAG_TREE_LEVELWISE if levelwise else 0
    A2 = A.view(b * m, n)
    rc = lib.tsqr_factor_batched(_dtype_code(A), b, m, n, _ptr(A2), n, _ptr(R), R.stride(1), R.stride(0),
                                 _opts(0, chains, arity, flags), ctypes.byref(h) if want_q else None, _stream(A))
    _lib.check("tsqr_factor_batched", rc)
    return R, (QTree(h, A2, b * m, n) if want_q else None)


def sign_normalize_batched(Q: torch.Tensor | None, R: torch.Tensor):
    """Per member b: R_b <- D_b R_b, Q_b <- Q_b D_b (Q: [batch, m, n] or its
    stacked 2-D view; R: [batch, n, n]), D_b = sign(diag R_b), in place."""
    lib = _lib.load()
    b, n = R.shape[0], R.shape[1]
    m = (Q.numel() // (b * n)) if Q is not None else n
    ldq = n
    rc = lib.tsqr_sign_normalize_batched(_dtype_code(R), b, m, n, _ptr(Q) if Q is not None else None, ldq,
                                         _ptr(R), R.stride(1), R.stride(0), _stream(R))
    _lib.check("tsqr_sign_normalize_batched", rc)
    return Q, R


def lstsq(A: torch.Tensor, B: torch.Tensor, rnorm: bool = True, block_rows=0, chains=0, arity=0):
    """Least squares min ||A X - B|| column by column (A m x n of full column
    rank, m >= n, n <= 64; B m x k or a vector of m).  Returns (X, rnorm):
    X n x k (or n), rnorm the k residual norms (or None).  A and B are not
    modified: the library works on copies (tsqr_lstsq overwrites both)."""
    lib = _lib.load()
    m, n = A.shape
    if B.dtype != A.dtype or B.device != A.device or B.size(0) != m:
        raise ValueError("B must be an m x k (or m) tensor of A's dtype and device")
    vec = B.dim() == 1
    W = A.contiguous().clone()
    Bw = (B.reshape(m, 1) if vec else B).contiguous().clone()
    k = Bw.size(1)
    rn = torch.empty(k, dtype=A.dtype, device=A.device) if rnorm and k > 0 else None
    rc = lib.tsqr_lstsq(_dtype_code(A), m, n, _ptr(W), _ld(W), k, _ptr(Bw), max(k, 1),
                        _ptr(rn) if rn is not None else None, _opts(block_rows, chains, arity), _stream(A))
    _lib.check("tsqr_lstsq", rc)
    X = Bw[:n]
    if vec:
        return X[:, 0], (rn[0] if rn is not None else None)
    return X, rn


def cholqr(A: torch.Tensor, passes: int = 1, out_q: torch.Tensor | None = None):
    """CholeskyQR (passes = 1) or CholeskyQR2 (passes = 2) of A (m x n,
    n <= 64), for comparison with TSQR: returns (Q, R), diag(R) > 0.  A is not
    modified unless out_q is A."""
    lib = _lib.load()
    m, n = A.shape
    Q = out_q if out_q is not None else torch.empty(m, n, dtype=A.dtype, device=A.device)
    R = torch.empty(n, n, dtype=A.dtype, device=A.device)
    rc = lib.tsqr_cholqr(_dtype_code(A), m, n, _ptr(A), _ld(A), _ptr(Q), _ld(Q), _ptr(R), _ld(R), int(passes),
                         _stream(A))
    _lib.check("tsqr_cholqr", rc)
    return Q, R


def mgs(A: torch.Tensor, out_q: torch.Tensor | None = None):
    """Modified Gram-Schmidt of A (m x n, n <= 64), for comparison with TSQR:
    returns (Q, R), diag(R) > 0.  A is not modified unless out_q is A."""
    lib = _lib.load()
    m, n = A.shape
    Q = out_q if out_q is not None else torch.empty(m, n, dtype=A.dtype, device=A.device)
    R = torch.empty(n, n, dtype=A.dtype, device=A.device)
    rc = lib.tsqr_mgs(_dtype_code(A), m, n, _ptr(A), _ld(A), _ptr(Q), _ld(Q), _ptr(R), _ld(R), _stream(A))
    _lib.check("tsqr_mgs", rc)
    return Q, R


def sign_normalize(Q: torch.Tensor | None, R: torch.Tensor):
    """R <- D R, Q <- Q D with D = sign(diag R), sign(0) = +1 (in place)."""
    lib = _lib.load()
    n = R.size(0)
    m = Q.size(0) if Q is not None else n
    rc = lib.tsqr_sign_normalize(_dtype_code(R), m, n, _ptr(Q) if Q is not None else None,
                                 _ld(Q) if Q is not None else n, _ptr(R), _ld(R), _stream(R))
    _lib.check("tsqr_sign_normalize", rc)
    return Q, R


def caqr(A: torch.Tensor, panel: int = 64, update=None, block_rows=0, chains=0, arity=0, shared_cus=False):
    """CAQR of A (m x n, m >= n), IN PLACE.  `update` is the dtype of the
    trailing-update arithmetic (default: A's dtype; torch.float32 with a
    float64 A gives the mixed-precision update).  shared_cus: panels and
    updates on every compute unit (TSQR_FLAG_SHARED_CUS) instead of a few
    units per XCD reserved for the panels; same bits.  Returns (R, QTree)
    with R the upper triangle of A's first n rows (a copy)."""
    lib = _lib.load()
    m, n = A.shape
    upd = _dtype_code(A) if update is None else (_lib.TSQR_F64 if update == torch.float64 else _lib.TSQR_F32)
    h = ctypes.c_void_p()
    rc = lib.caqr_factor(_dtype_code(A), m, n, _ptr(A), _ld(A), panel, upd,
                         _opts(block_rows, chains, arity, _lib.TSQR_FLAG_SHARED_CUS if shared_cus else 0),
                         ctypes.byref(h), _stream(A))
    _lib.check("caqr_factor", rc)
    R = torch.empty(n, n, dtype=A.dtype, device=A.device)
    _lib.check("tsqr_copy_r", lib.tsqr_copy_r(_dtype_code(A), n, _ptr(A), _ld(A), _ptr(R), _ld(R), _stream(A)))
    return R, QTree(h, A, m, n)


def caqr_left(A: torch.Tensor, panel: int = 64, block_cols: int = 0, update=None, chains=0):
    """Left-looking CAQR of A (m x n, m >= n) over column blocks of
    `block_cols` columns (0 = the panel width: plain left-looking), IN
    PLACE; same output layout and implicit Q as caqr.  Returns (R, QTree)."""
    lib = _lib.load()
    m, n = A.shape
    upd = _dtype_code(A) if update is None else (_lib.TSQR_F64 if update == torch.float64 else _lib.TSQR_F32)
    h = ctypes.c_void_p()
    rc = lib.caqr_factor_left(_dtype_code(A), m, n, _ptr(A), _ld(A), panel, block_cols, upd,
                              _opts(0, chains, 0, 0), ctypes.byref(h), _stream(A))
    _lib.check("caqr_factor_left", rc)
    R = torch.empty(n, n, dtype=A.dtype, device=A.device)
    _lib.check("tsqr_copy_r", lib.tsqr_copy_r(_dtype_code(A), n, _ptr(A), _ld(A), _ptr(R), _ld(R), _stream(A)))
    return R, QTree(h, A, m, n)


def qr(A: torch.Tensor, block_rows=0, chains=0, arity=0):
    """Thin QR with diag(R) >= 0; A is not modified.  Returns (Q, R)."""
    W = A.contiguous().clone()
    R, qt = factor(W, block_rows=block_rows, chains=chains, arity=arity)
    Q = qt.form_q_signed(R)
    qt.close()
    return Q, R


def qr_backward(Q: torch.Tensor, R: torch.Tensor, dQ: torch.Tensor | None, dR: torch.Tensor | None) -> torch.Tensor:
    """dA for the sign-normalised thin QR (2-D, or batched 3-D tensors)."""
    lib = _lib.load()
    batched = Q.dim() == 3
    Qb = Q if batched else Q.unsqueeze(0)
    Rb = R if batched else R.unsqueeze(0)
    B, m, n = Qb.shape
    dQb = None if dQ is None else (dQ if batched else dQ.unsqueeze(0)).contiguous()
    dRb = None if dR is None else (dR if batched else dR.unsqueeze(0)).contiguous()
    Qb = Qb.contiguous()
    Rb = Rb.contiguous()
    dA = torch.empty_like(Qb)
    rc = lib.tsqr_backward(_dtype_code(Qb), B, m, n, _ptr(Qb), n, m * n, _ptr(Rb), n, n * n,
                           _ptr(dQb) if dQb is not None else None, n, m * n,
                           _ptr(dRb) if dRb is not None else None, n, n * n,
                           _ptr(dA), n, m * n, _stream(Qb))
    _lib.check("tsqr_backward", rc)
    return dA if batched else dA[0]


class TSQRFunction(torch.autograd.Function):
    """A -> (Q, R), thin QR with diag(R) >= 0 by TSQR; backward by the QR
    adjoint kernels (no stored reflectors).  A may be 2-D or a 3-D batch."""

    @staticmethod
    def forward(ctx, A, block_rows=0, chains=0, arity=0):
        batched = A.dim() == 3
        As = A.detach().contiguous()
        if batched:
            # one factorisation of the whole batch (a forest of trees), then
            # every member's explicit Q in one pass
            W = As.clone()
            R, qt = factor_batched(W, chains=chains, arity=arity)
            Q = qt.form_q_signed(R)
            qt.close()
            Q = Q.view(As.shape)
        else:
            Q, R = qr(As, block_rows=block_rows, chains=chains, arity=arity)
        ctx.save_for_backward(Q, R)
        return Q, R

    @staticmethod
    def backward(ctx, dQ, dR):
        Q, R = ctx.saved_tensors
        dA = qr_backward(Q, R, dQ, dR)
        return dA, None, None, None


def tsqr(A: torch.Tensor, block_rows=0, chains=0, arity=0):
    """Differentiable thin QR (Q, R) with diag(R) >= 0."""
    return TSQRFunction.apply(A, block_rows, chains, arity)


class BatchPlan:
    """Batched TSQR of many uneven matrices in one graph launch.

    shapes: list of (m, n); opts: None (library defaults) or a list of
    (chains, arity) per matrix (0 = default), e.g. from
    ``autotune.choose_batch``.  The device arrays of matrix pointers and
    leading dimensions live in the plan, so repeated ``factor`` calls replay
    the same captured graph with new matrices.
    """

    def __init__(self, shapes, dtype=torch.float64, opts=None, device="cuda"):
        lib = _lib.load()
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.count = len(self.shapes)
        self.dtype = dtype
        self.device = torch.device(device)
        code = _lib.TSQR_F64 if dtype == torch.float64 else _lib.TSQR_F32
        ms = (ctypes.c_int64 * self.count)(*[m for m, _ in self.shapes])
        ns = (ctypes.c_int64 * self.count)(*[n for _, n in self.shapes])
        popts = None
        if opts is not None:
            arr = (_lib.TsqrOpts * self.count)()
            for i, (chains, arity) in enumerate(opts):
                arr[i] = _lib.opts(0, int(chains), int(arity))
            popts = arr
        self._h = ctypes.c_void_p()
        _lib.check("tsqr_batch_plan_create", lib.tsqr_batch_plan_create(code, self.count, ms, ns, popts,
                                                                         ctypes.byref(self._h)))
        # device argument arrays (stable addresses for graph replay)
        self._dA = torch.zeros(self.count, dtype=torch.int64, device=self.device)
        self._dlda = torch.zeros(self.count, dtype=torch.int64, device=self.device)
        self._dR = torch.zeros(self.count, dtype=torch.int64, device=self.device)
        self._dldr = torch.zeros(self.count, dtype=torch.int64, device=self.device)

    def info(self) -> dict:
        out = (ctypes.c_int64 * 6)()
        _lib.check("tsqr_batch_plan_info", _lib.load().tsqr_batch_plan_info(self._h, out))
        keys = ("count", "chains", "classes", "workspace_bytes", "graph_captured", "workers")
        return dict(zip(keys, (int(v) for v in out)))

    def factor(self, As, Rs=None):
        """Factor the matrices As (list of device tensors, in place: each is
        overwritten with its reflectors).  Returns the list of R factors
        (n x n, diag(R) with the Householder signs)."""
        if len(As) != self.count:
            raise ValueError("expected %d matrices" % self.count)
        if Rs is None:
            Rs = [torch.empty(n, n, dtype=self.dtype, device=self.device) for _, n in self.shapes]
        for A, (m, n) in zip(As, self.shapes):
            if A.shape != (m, n) or A.dtype != self.dtype:
                raise ValueError("matrix shape/dtype does not match the plan")
        ha = torch.tensor([A.data_ptr() for A in As], dtype=torch.int64)
        hl = torch.tensor([_ld(A) for A in As], dtype=torch.int64)
        hr = torch.tensor([R.data_ptr() for R in Rs], dtype=torch.int64)
        hlr = torch.tensor([_ld(R) for R in Rs], dtype=torch.int64)
        self._dA.copy_(ha)
        self._dlda.copy_(hl)
        self._dR.copy_(hr)
        self._dldr.copy_(hlr)
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _lib.check("tsqr_batch_factor", _lib.load().tsqr_batch_factor(
            self._h, _ptr(self._dA), _ptr(self._dlda), _ptr(self._dR), _ptr(self._dldr), st))
        return Rs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().tsqr_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
