"""GPU parity of left-looking CAQR over column blocks (caqr_factor_left,
Sec. 3.2) against the oracle and against right-looking CAQR.

Each column receives the same panel transformations in the same order as in
right-looking CAQR, so R agrees with the oracle to the FP64 gates of the
right-looking tests (normwise R error <= 1e-11, backward error and
orthogonality <= 1e-13) and with caqr_factor's R to rounding.  Cases: plain
left-looking (blocks of one panel), blocks of several panels, a ragged last
block and panel, one block wider than n (right-looking without look-ahead),
FP32 products on FP64 storage and FP32 storage.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)


def _backward_error(qt, A_dev, R, m, n):
    X = torch.zeros(m, n, dtype=A_dev.dtype, device="cuda")
    X[:n] = R
    qt.apply_q(X)
    return (torch.linalg.norm((X - A_dev).double()) / torch.linalg.norm(A_dev.double())).item()


def _oracle_r(A):
    YR = oracle.geqrf_blocked(A, 64)[0] if A.shape[0] >= 2048 else oracle.geqrf(A)[0]
    R = oracle.r_of(YR)
    return R * oracle.signs(R)[:, None]


def _signed(R):
    Rg = R.double().cpu().numpy()
    return Rg * oracle.signs(Rg)[:, None]


@pytest.mark.parametrize("m,n,panel,block", [(1000, 1000, 64, 64), (3000, 700, 64, 256), (513, 200, 16, 48),
                                             (2048, 1024, 64, 4096), (2049, 130, 64, 0)])
def test_caqr_left_f64(m, n, panel, block):
    import paper_0808_2664_amd as tq
    _note("case: caqr_left f64 m=%d n=%d panel=%d block_cols=%d" % (m, n, panel, block))
    A = workloads.gaussian(m, n, 500 + m + n)
    Ad = _dev(A)
    A_keep = Ad.clone()
    R, qt = tq.caqr_left(Ad, panel=panel, block_cols=block)
    torch.cuda.synchronize()
    info = qt.info()
    assert info["kind"] == 1 and info["panel"] == panel
    Ro = _oracle_r(A)
    e = oracle.rel_err(_signed(R), Ro)
    be = _backward_error(qt, A_keep, R, m, n)
    Q = qt.form_q().cpu().numpy()
    orth = oracle.orthogonality(Q)
    qt.close()
    # right-looking CAQR of the same matrix
    Ad2 = _dev(A)
    R2, qt2 = tq.caqr(Ad2, panel=panel)
    torch.cuda.synchronize()
    qt2.close()
    e_rl = oracle.rel_err(_signed(R), _signed(R2))
    _note("  R error vs oracle %.2e, vs right-looking %.2e; backward error %.2e; orthogonality %.2e"
          % (e, e_rl, be, orth))
    assert e <= 1e-11 and e_rl <= 1e-11
    assert be <= 1e-13 and orth <= 1e-13


def test_caqr_left_f32_products_on_f64_storage():
    import paper_0808_2664_amd as tq
    _note("case: caqr_left fp32 products 1024^2, blocks of 256")
    A = workloads.gaussian(1024, 1024, 78)
    Ad = _dev(A)
    A_keep = Ad.clone()
    R, qt = tq.caqr_left(Ad, panel=64, block_cols=256, update=torch.float32)
    torch.cuda.synchronize()
    e = oracle.rel_err(_signed(R), _oracle_r(A))
    be = _backward_error(qt, A_keep, R, 1024, 1024)
    qt.close()
    _note("  R error %.2e, backward error %.2e" % (e, be))
    assert 1e-12 < e <= 1e-4      # the FP32 products really ran
    assert be <= 1e-4


def test_caqr_left_f32_storage():
    import paper_0808_2664_amd as tq
    _note("case: caqr_left f32 storage 1200 x 500, blocks of 128")
    A = workloads.gaussian(1200, 500, 92).astype(np.float32)
    Ad = _dev(A, torch.float32)
    A_keep = Ad.clone()
    R, qt = tq.caqr_left(Ad, panel=64, block_cols=128)
    torch.cuda.synchronize()
    e = oracle.rel_err(_signed(R), _oracle_r(A.astype(np.float64)))
    be = _backward_error(qt, A_keep, R, 1200, 500)
    qt.close()
    _note("  R error %.2e, backward error %.2e" % (e, be))
    assert e <= 5e-4 and be <= 1e-5


def test_caqr_left_4096_blocks_of_2048_both_updates():
    """4096 x 4096 in column blocks of 2048: the earlier panels' Q^T reach the
    second block through the wide apply kernels (asserted on the first panel's
    tree: 8 chains x 32 column groups of 64);
    the whole R against the oracle's blocked Householder QR, FP64 update and
    FP32 products."""
    import paper_0808_2664_amd as tq
    N = 4096
    A = workloads.gaussian(N, N, 960)
    Ro = _oracle_r(A)
    for upd in (torch.float64, torch.float32):
        _note("case: caqr_left 4096^2 blocks of 2048, update %s" % upd)
        Ad = _dev(A)
        A_keep = Ad.clone()
        R, qt = tq.caqr_left(Ad, panel=64, block_cols=2048, update=upd)
        torch.cuda.synchronize()
        assert qt.wide_layout(2048, panel=0)
        e = oracle.rel_err(_signed(R), Ro)
        be = _backward_error(qt, A_keep, R, N, N)
        qt.close()
        _note("  R error %.2e, backward error %.2e" % (e, be))
        if upd == torch.float64:
            assert e <= 1e-11 and be <= 1e-13
        else:
            assert 1e-12 < e <= 1e-4 and be <= 1e-4
