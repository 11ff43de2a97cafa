"""Batched TSQR of stacked independent matrices (tsqr_factor_batched): each
member is reduced on its own tree, so every member's R, explicit Q and
Q^T B equal, bit for bit, those of tsqr_factor on that member alone with the
same chains per member; and they match the oracle."""
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


@pytest.mark.parametrize("batch,m,n,chains,levelwise", [(5, 3000, 20, 4, False), (3, 4100, 64, 8, True),
                                                        (4, 777, 7, 2, False)])
def test_forest_equals_single_calls_bitwise(batch, m, n, chains, levelwise):
    import paper_0808_2664_amd as tq
    _note("case: forest %d x %d x %d chains %d levelwise %s" % (batch, m, n, chains, levelwise))
    A = np.stack([workloads.gaussian(m, n, 600 + b) for b in range(batch)])
    B = np.stack([workloads.gaussian(m, 5, 700 + b) for b in range(batch)])
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda().view(batch * m, 5)
    R, qt = tq.factor_batched(Ad, chains=chains, levelwise=levelwise)
    Q = qt.form_q()
    qt.apply_qt(Bd)
    torch.cuda.synchronize()
    for b in range(batch):
        Ab = torch.from_numpy(A[b]).cuda()
        Bb = torch.from_numpy(B[b]).cuda()
        Rb, qb = tq.factor(Ab, chains=chains, levelwise=levelwise)
        Qb = qb.form_q()
        qb.apply_qt(Bb)
        torch.cuda.synchronize()
        assert torch.equal(R[b], Rb)
        assert torch.equal(Q[b * m:(b + 1) * m], Qb)
        assert torch.equal(Bd[b * m:(b + 1) * m], Bb)
        qb.close()
        Qo, Ro = oracle.qr(A[b])
        Rg = Rb.cpu().numpy()
        d = oracle.signs(Rg)
        assert oracle.rel_err(Rg * d[:, None], Ro) <= 1e-11
        assert oracle.rel_err(Qb.cpu().numpy() * d[None, :], Qo) <= 1e-11
    qt.close()


@pytest.mark.parametrize("batch,m,n,dt", [(7, 1000, 33, torch.float64), (300, 128, 16, torch.float64),
                                          (40, 2048, 64, torch.float32)])
def test_forest_default_chains_against_oracle(batch, m, n, dt):
    import paper_0808_2664_amd as tq
    _note("case: forest default chains %d x %d x %d %s" % (batch, m, n, dt))
    A = np.stack([workloads.gaussian(m, n, 800 + b) for b in range(batch)])
    if dt == torch.float32:
        A = A.astype(np.float32)
    Ad = torch.from_numpy(A).cuda()
    R, qt = tq.factor_batched(Ad)
    Q = qt.form_q()
    tq.sign_normalize_batched(Q, R)
    torch.cuda.synchronize()
    gate = 1e-11 if dt == torch.float64 else 1e-5
    Rg, Qg = R.double().cpu().numpy(), Q.double().cpu().numpy().reshape(batch, m, n)
    for b in range(batch):
        Qo, Ro = oracle.qr(A[b].astype(np.float64))
        assert np.all(np.diag(Rg[b]) >= 0)
        assert oracle.rel_err(Rg[b], Ro) <= gate
        assert oracle.rel_err(Qg[b], Qo) <= gate
    qt.close()
