"""GPU parity of tsqr_lstsq (least squares through TSQR, Q^T B and back
substitution) against the oracle's least squares.

Gates: FP64 X and residual norms within max(1e-12, 100 cond^2 u)
(normwise, relative; the solution's sensitivity grows like cond^2 u for a
nonzero residual), and 1e-9 for the constructed cond 1e3 case; FP32 within
5e-4.  At the full 2^20 x 64 size the
oracle solves two sampled columns, and every column is checked through
properties that hold at any size: the residual is orthogonal to range(A) and
its norm equals the reported one.
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_0808_2664_amd.tsqr import lstsq

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)


def _rel(x, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(x, np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))


def test_lstsq_hand_3x2():
    g = json.load(open(os.path.join(GOLD, "householder_3x2.json")))
    A = np.array([[float(Fraction(v)) for v in r] for r in g["A"]])
    b = np.array([float(Fraction(v)) for v in g["b"]])
    _note("lstsq hand 3x2")
    x, rn = lstsq(_dev(A), _dev(b))
    torch.cuda.synchronize()
    np.testing.assert_allclose(x.cpu().numpy(), [4 / 9, 1 / 9], rtol=0, atol=1e-15)
    assert abs(float(rn) - 1 / 3) < 1e-15


@pytest.mark.parametrize("m,n,k,opts", [
    (5000, 16, 7, {}),
    (70001, 64, 33, {}),                 # ragged rows; the wide apply path (k > 32)
    (4096, 8, 1, {}),
    (1000, 64, 64, {}),
    (64, 64, 3, {}),                     # square: no residual rows
    (65, 64, 20, {}),
    (200000, 32, 5, {"chains": 7, "arity": 3}),
    (300000, 64, 32, {"chains": 100}),
])
def test_lstsq_f64_matches_oracle(m, n, k, opts):
    A = workloads.gaussian(m, n, 1000 + n + k)
    if m == n:
        A = A + 8 * np.eye(n)
    B = workloads.gaussian(m, k, 2000 + n + k)
    _note("lstsq f64 m=%d n=%d k=%d %s" % (m, n, k, opts))
    X, rn = lstsq(_dev(A), _dev(B), **opts)
    torch.cuda.synchronize()
    Xo, rno = oracle.lstsq(A, B)
    # near-square Gaussians are less well conditioned: widen the gate to
    # 100 cond^2 u where that exceeds 1e-12
    sv = np.linalg.svd(A, compute_uv=False)
    tol = max(1e-12, 100 * (sv[0] / sv[-1]) ** 2 * np.finfo(np.float64).eps / 2)
    assert _rel(X.cpu().numpy(), Xo) <= tol
    if m > n:
        assert _rel(rn.cpu().numpy(), rno) <= tol
    else:
        assert float(rn.abs().max()) == 0.0


def test_lstsq_f64_cond_1e3():
    m, n, k = 20000, 32, 4
    A = workloads.conditioned(m, n, 1e3, 31, 32)
    B = workloads.gaussian(m, k, 33)
    _note("lstsq f64 cond 1e3")
    X, rn = lstsq(_dev(A), _dev(B))
    torch.cuda.synchronize()
    Xo, rno = oracle.lstsq(A, B)
    assert _rel(X.cpu().numpy(), Xo) <= 1e-9
    assert _rel(rn.cpu().numpy(), rno) <= 1e-12


@pytest.mark.parametrize("m,n,k", [(20000, 32, 4), (4097, 64, 40), (1000, 8, 1)])
def test_lstsq_f32_matches_oracle(m, n, k):
    # inputs drawn in FP64 and rounded; the oracle runs on the rounded values
    A = workloads.gaussian(m, n, 3000 + n).astype(np.float32)
    B = workloads.gaussian(m, k, 3100 + n).astype(np.float32)
    _note("lstsq f32 m=%d n=%d k=%d" % (m, n, k))
    X, rn = lstsq(_dev(A, torch.float32), _dev(B, torch.float32))
    torch.cuda.synchronize()
    Xo, rno = oracle.lstsq(A.astype(np.float64), B.astype(np.float64))
    assert _rel(X.cpu().numpy(), Xo) <= 5e-4
    assert _rel(rn.cpu().numpy(), rno) <= 5e-4


def test_lstsq_without_rhs_and_without_rnorm():
    A = workloads.gaussian(3000, 16, 41)
    B = workloads.gaussian(3000, 3, 42)
    _note("lstsq k=0 and rnorm=False")
    X0, rn0 = lstsq(_dev(A), _dev(B[:, :0]))
    assert tuple(X0.shape) == (16, 0) and rn0 is None
    X, rn = lstsq(_dev(A), _dev(B), rnorm=False)
    torch.cuda.synchronize()
    assert rn is None
    Xo, _ = oracle.lstsq(A, B)
    assert _rel(X.cpu().numpy(), Xo) <= 1e-12


def test_lstsq_full_size_sampled_and_properties():
    # 2^20 x 64 FP64 with 32 right-hand sides, the benchmark's launch shape
    m, n, k = 1 << 20, 64, 32
    A = workloads.gaussian(m, n, 51)
    B = workloads.gaussian(m, k, 52)
    Ad, Bd = _dev(A), _dev(B)
    _note("lstsq full size 2^20 x 64, k = 32")
    X, rn = lstsq(Ad, Bd)
    torch.cuda.synchronize()
    # properties for every column: A^T r = 0 and ||r|| = rnorm
    Rs = Ad @ X - Bd
    ortho = torch.linalg.norm(Ad.T @ Rs) / (torch.linalg.norm(Ad) * torch.linalg.norm(Rs))
    # the check's own GEMMs sum 2^20 products per entry: ~sqrt(m) u of slack
    assert float(ortho) <= 1e-11
    rr = torch.linalg.norm(Rs, dim=0)
    assert float(torch.max(torch.abs(rr - rn) / rr)) <= 1e-12
    # two sampled columns against the oracle
    cols = [0, 29]
    Xo, rno = oracle.lstsq(A, B[:, cols])
    assert _rel(X[:, cols].cpu().numpy(), Xo) <= 1e-12
    assert _rel(rn[cols].cpu().numpy(), rno) <= 1e-12



def test_lstsq_single_column_closed_form():
    # n = 1: x = a^T b / a^T a, residual ||b - a x||
    a = workloads.gaussian(5000, 1, 61)
    B = workloads.gaussian(5000, 3, 62)
    _note("lstsq n = 1")
    X, rn = lstsq(_dev(a), _dev(B))
    torch.cuda.synchronize()
    x = (a[:, 0] @ B) / (a[:, 0] @ a[:, 0])
    np.testing.assert_allclose(X.cpu().numpy()[0], x, rtol=1e-12)
    np.testing.assert_allclose(rn.cpu().numpy(), np.linalg.norm(B - a @ x[None, :], axis=0), rtol=1e-12)


def test_lstsq_through_the_abi_with_padded_leading_dimensions():
    # lda > n and ldb > k: views into wider row-major buffers, called through the C ABI
    import ctypes

    from paper_0808_2664_amd import _lib
    m, n, k = 9000, 24, 5
    A = workloads.gaussian(m, n, 63)
    B = workloads.gaussian(m, k, 64)
    Aw = torch.zeros(m, n + 7, dtype=torch.float64, device="cuda")
    Bw = torch.zeros(m, k + 3, dtype=torch.float64, device="cuda")
    Aw[:, :n] = _dev(A)
    Bw[:, :k] = _dev(B)
    rn = torch.empty(k, dtype=torch.float64, device="cuda")
    _note("lstsq through the ABI, lda = n + 7, ldb = k + 3")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _lib.load().tsqr_lstsq(_lib.TSQR_F64, m, n, ctypes.c_void_p(Aw.data_ptr()), n + 7, k,
                                ctypes.c_void_p(Bw.data_ptr()), k + 3, ctypes.c_void_p(rn.data_ptr()), None, st)
    assert rc == 0
    torch.cuda.synchronize()
    Xo, rno = oracle.lstsq(A, B)
    assert _rel(Bw[:n, :k].cpu().numpy(), Xo) <= 1e-12
    assert _rel(rn.cpu().numpy(), rno) <= 1e-12
    # the padding columns are untouched
    assert float(Bw[:, k:].abs().max()) == 0.0
