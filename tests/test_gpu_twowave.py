"""The two-wave chain engine (FP64, more than 32 columns: two waves split a
chain's columns, then the tree in a second launch) against the one-wave
engine (TSQR_FLAG_ONE_WAVE): the same arithmetic in the same order, so R,
the reflectors, tau / T (through the explicit Q and Q^T B) are equal bit for
bit; and against the oracle."""
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


CASES = [
    # m, n, chains, levelwise
    (4096, 64, 0, False), (70000, 64, 0, False), (70000, 64, 7, True), (5000, 33, 0, False), (3000, 40, 3, False),
    (2500, 48, 0, True), (2049, 50, 0, False), (64, 64, 0, False), (129, 64, 1, False), (100000, 57, 0, False),
    (1 << 18, 64, 0, False),
]


@pytest.mark.parametrize("m,n,chains,levelwise", CASES)
def test_two_wave_equals_one_wave_bitwise(m, n, chains, levelwise):
    import paper_0808_2664_amd as tq
    _note("case: two-wave vs one-wave m=%d n=%d chains=%d levelwise=%s" % (m, n, chains, levelwise))
    A = workloads.gaussian(m, n, 1000 + m % 997 + n)
    B = workloads.gaussian(m, 9, 2000 + n)
    out = []
    for one_wave in (False, True):
        Ad = torch.from_numpy(A).cuda()
        R, qt = tq.factor(Ad, chains=chains, levelwise=levelwise, one_wave=one_wave)
        Q = qt.form_q()
        Bd = torch.from_numpy(B).cuda()
        qt.apply_qt(Bd)
        Rr, _ = tq.factor(torch.from_numpy(A).cuda(), chains=chains, levelwise=levelwise, one_wave=one_wave,
                          want_q=False)
        torch.cuda.synchronize()
        out.append((R.clone(), Ad.clone(), Q, Bd, Rr))
        qt.close()
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    Qo, Ro = oracle.qr(A)
    Rg = out[0][0].cpu().numpy()
    d = oracle.signs(Rg)
    assert oracle.rel_err(Rg * d[:, None], Ro) <= 1e-11
    assert oracle.rel_err(out[0][2].cpu().numpy() * d[None, :], Qo) <= 1e-11
