"""Status word of the bounded waits in the panel-pipelined tree.

In the pipelined tree a wave waits for its children's progress with a
bounded poll (tsqr_opts.max_polls).  A wave that gives up must not hang or
fault: it finishes with whatever rows are in memory, and the give-up is
reported by tsqr_check_status as TSQR_ERR_TIMEOUT.  The condition is forced
from the host with a one-poll bound on a tree whose last chain is 16 times
shorter than its sibling, so its node wave polls before the sibling is done;
every kernel still ends normally.
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=torch.float64)


def test_normal_factor_reports_success():
    import paper_0808_2664_amd as tq
    from paper_0808_2664_amd import _lib
    _note("case: status after a normal pipelined factor 65536 x 64")
    assert tq.check_status() in (0, _lib.TSQR_ERR_TIMEOUT)  # clears anything left by earlier tests
    A = workloads.gaussian(65536, 64, 901)
    R, _ = tq.factor(_dev(A), want_q=False)
    assert tq.check_status() == 0
    Ro = oracle.qr(A)[1]
    Rg = R.cpu().numpy()
    assert oracle.rel_err(Rg * oracle.signs(Rg)[:, None], Ro) <= 1e-11


def test_wait_give_up_is_reported_and_cleared():
    import paper_0808_2664_amd as tq
    from paper_0808_2664_amd import _lib
    m, n, chains = 64 * (16 * 63 + 1), 64, 64
    geo = tq.plan_geometry(m, n, chains=chains)
    assert geo["chains"] == 64 and geo["chain_rows"] == 1024 and m - 63 * 1024 == 64
    A = workloads.gaussian(m, n, 902)
    _note("case: one-poll waits, %d x %d, %d chains (last chain one block)" % (m, n, chains))
    tq.check_status()
    R, _ = tq.factor(_dev(A), chains=chains, want_q=False, max_polls=1)
    assert tq.check_status() == _lib.TSQR_ERR_TIMEOUT
    assert tq.check_status() == 0  # read and cleared
    _note("case: the same factor with the default bound")
    R, qt = tq.factor(_dev(A), chains=chains)
    assert tq.check_status() == 0
    Ro = oracle.qr(A)[1]
    Rg = R.cpu().numpy()
    assert oracle.rel_err(Rg * oracle.signs(Rg)[:, None], Ro) <= 1e-11
    qt.close()
