"""GPU parity of tsqr_cholqr (CholeskyQR and CholeskyQR2, the comparison
algorithms of Sec. 2.3) against the oracle's CholeskyQR.

Gates: FP64 Q and R within 1e-12 (normwise, relative) of the oracle on
well-conditioned inputs (Gaussian); FP32 within 5e-4.  Conditioning is the
point of the comparison, so it is checked as a property: at cond 1e7 one pass
loses orthogonality (of order cond^2 u) on the GPU as in the oracle, the
second pass restores it, and TSQR on the same input keeps it.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_0808_2664_amd.tsqr import cholqr, qr

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)


@pytest.mark.parametrize("m,n,passes", [(5000, 16, 1), (70001, 64, 1), (4096, 8, 2), (100003, 32, 2),
                                        (64, 64, 1), (1 << 20, 64, 1)])
def test_cholqr_f64_matches_oracle(m, n, passes):
    A = workloads.gaussian(m, n, 4000 + n + passes)
    if m == n:
        A = A + 8 * np.eye(n)
    _note("cholqr f64 m=%d n=%d passes=%d" % (m, n, passes))
    Q, R = cholqr(_dev(A), passes)
    torch.cuda.synchronize()
    if m > 200000:
        # full size: sampled rows of Q (the oracle's Q row i needs only A's row i and R)
        Qo, Ro = oracle.cholqr(A, passes)
        rows = np.r_[0:64, m // 2:m // 2 + 64, m - 64:m]
        assert oracle.rel_err(R.cpu().numpy(), Ro) <= 1e-12
        assert oracle.rel_err(Q[rows].cpu().numpy(), Qo[rows]) <= 1e-12
        return
    Qo, Ro = oracle.cholqr(A, passes)
    assert oracle.rel_err(R.cpu().numpy(), Ro) <= 1e-12
    assert oracle.rel_err(Q.cpu().numpy(), Qo) <= 1e-12
    assert float(torch.tril(R, -1).abs().max()) == 0.0


@pytest.mark.parametrize("m,n,passes", [(20000, 32, 1), (4097, 64, 2)])
def test_cholqr_f32_matches_oracle(m, n, passes):
    A = workloads.gaussian(m, n, 4100 + n).astype(np.float32)
    _note("cholqr f32 m=%d n=%d passes=%d" % (m, n, passes))
    Q, R = cholqr(_dev(A, torch.float32), passes)
    torch.cuda.synchronize()
    Qo, Ro = oracle.cholqr(A.astype(np.float64), passes)
    assert oracle.rel_err(R.cpu().numpy(), Ro) <= 5e-4
    assert oracle.rel_err(Q.cpu().numpy(), Qo) <= 5e-4


def test_cholqr_conditioning_against_tsqr():
    m, n = 20000, 16
    A = workloads.conditioned(m, n, 1e7, 71, 72)
    Ad = _dev(A)
    _note("cholqr cond 1e7: one pass, two passes, TSQR")
    Q1, _ = cholqr(Ad, 1)
    Q2, R2 = cholqr(Ad, 2)
    Qt, Rt = qr(Ad)
    torch.cuda.synchronize()
    o1 = oracle.orthogonality(Q1.cpu().numpy())
    o2 = oracle.orthogonality(Q2.cpu().numpy())
    ot = oracle.orthogonality(Qt.cpu().numpy())
    o1_orc = oracle.orthogonality(oracle.cholqr(A, 1)[0])
    assert o1 > 1e-6 and o1_orc > 1e-6          # one pass: ~cond^2 u
    assert o2 < 1e-13 and ot < 1e-13            # CholeskyQR2 and TSQR keep orthogonality
    assert oracle.residual(A, Q2.cpu().numpy(), R2.cpu().numpy()) < 1e-14
    # both are QR factorisations of A: R agrees with TSQR's (diag >= 0) to ~cond u
    assert oracle.rel_err(R2.cpu().numpy(), Rt.cpu().numpy()) < 1e-8


def test_cholqr_in_place():
    A = workloads.gaussian(30000, 32, 81)
    Ad = _dev(A)
    _note("cholqr in place (Q = A), two passes")
    Q, R = cholqr(Ad, 2, out_q=Ad)
    torch.cuda.synchronize()
    Qo, Ro = oracle.cholqr(A, 2)
    assert oracle.rel_err(Q.cpu().numpy(), Qo) <= 1e-12
    assert oracle.rel_err(R.cpu().numpy(), Ro) <= 1e-12


def test_cholqr_single_column_closed_form():
    # n = 1: R = ||a||, Q = a / ||a||
    a = workloads.gaussian(7000, 1, 91)
    _note("cholqr n = 1")
    Q, R = cholqr(_dev(a), 2)
    torch.cuda.synchronize()
    nrm = np.linalg.norm(a)
    assert abs(float(R[0, 0]) - nrm) <= 1e-13 * nrm
    np.testing.assert_allclose(Q.cpu().numpy(), a / nrm, rtol=0, atol=1e-15)


def test_cholqr_through_the_abi_with_padded_leading_dimensions():
    import ctypes

    from paper_0808_2664_amd import _lib
    m, n = 12000, 40
    A = workloads.gaussian(m, n, 92)
    Aw = torch.zeros(m, n + 5, dtype=torch.float64, device="cuda")
    Aw[:, :n] = _dev(A)
    Qw = torch.zeros(m, n + 3, dtype=torch.float64, device="cuda")
    Rw = torch.zeros(n, n + 9, dtype=torch.float64, device="cuda")
    _note("cholqr through the ABI, lda = n + 5, ldq = n + 3, ldr = n + 9")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _lib.load().tsqr_cholqr(_lib.TSQR_F64, m, n, ctypes.c_void_p(Aw.data_ptr()), n + 5,
                                 ctypes.c_void_p(Qw.data_ptr()), n + 3, ctypes.c_void_p(Rw.data_ptr()), n + 9, 2, st)
    assert rc == 0
    torch.cuda.synchronize()
    Qo, Ro = oracle.cholqr(A, 2)
    assert oracle.rel_err(Qw[:, :n].cpu().numpy(), Qo) <= 1e-12
    assert oracle.rel_err(Rw[:, :n].cpu().numpy(), Ro) <= 1e-12
    assert float(Qw[:, n:].abs().max()) == 0.0 and float(Rw[:, n:].abs().max()) == 0.0
