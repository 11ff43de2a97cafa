"""GPU parity of the batched TSQR (one graph launch over uneven matrices).

Every R is compared with the oracle after sign normalisation (normwise R
error <= 1e-11 in FP64, <= 5e-4 in FP32); the batched R must also equal,
bit for bit, the R of a single-matrix tsqr_factor with the same tree shape
(the same engine and the same arithmetic order).
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


def _shapes(count, seed, m_lo, m_hi, n_max=64):
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.integers(1, n_max + 1, size=count)
    return [(int(m), int(min(n, m))) for m, n in zip(ms, ns)]


def _r_err(R, A64):
    Rn = R * oracle.signs(R)[:, None]
    Ro = oracle.qr(A64)[1]
    return oracle.rel_err(Rn, Ro)


def test_batched_mixed_f64_matches_oracle_and_single_calls():
    import paper_0808_2664_amd as tq
    from paper_0808_2664_amd import autotune
    shapes = _shapes(60, 31, 64, 6000) + [(64, 64), (65, 64), (1, 1), (7, 3), (20000, 64), (4096, 16)]
    _note("case: batched f64, %d mixed shapes" % len(shapes))
    opts = autotune.choose_batch(shapes, torch.float64)
    As = [workloads.gaussian(m, n, 500 + i) for i, (m, n) in enumerate(shapes)]
    dev = [torch.from_numpy(a).cuda() for a in As]
    plan = tq.BatchPlan(shapes, torch.float64, opts=opts)
    Rs = plan.factor(dev)
    torch.cuda.synchronize()
    info = plan.info()
    assert info["count"] == len(shapes) and info["graph_captured"] == 1
    worst = 0.0
    for i, (A, R) in enumerate(zip(As, Rs)):
        e = _r_err(R.cpu().numpy(), A)
        worst = max(worst, e)
        assert e <= 1e-11, (i, shapes[i], e)
    _note("  worst R error %.2e" % worst)
    # bitwise equal to single-matrix factorisations with the same tree shape
    # (R only, as the batch), and equal to rounding to the Q-keeping ones
    for i in [0, 5, 17, 60, 61, 62, 63, 64, 65]:
        A1 = torch.from_numpy(As[i]).cuda()
        R1, none = tq.factor(A1, chains=opts[i][0], arity=opts[i][1], want_q=False)
        A2 = torch.from_numpy(As[i]).cuda()
        R2, qt = tq.factor(A2, chains=opts[i][0], arity=opts[i][1])
        torch.cuda.synchronize()
        assert none is None
        assert torch.equal(R1, Rs[i]), i
        assert torch.equal(A1, dev[i]), i       # the same reflectors in place
        assert torch.linalg.norm(R2 - R1).item() <= 1e-14 * torch.linalg.norm(R1).item(), i
        qt.close()
    plan.close()


def test_batched_graph_replay_and_recapture():
    import paper_0808_2664_amd as tq
    _note("case: batched replay")
    shapes = _shapes(24, 32, 100, 3000)
    plan = tq.BatchPlan(shapes, torch.float64)
    for rep in range(3):
        As = [workloads.gaussian(m, n, 900 + 31 * rep + i) for i, (m, n) in enumerate(shapes)]
        dev = [torch.from_numpy(a).cuda() for a in As]
        Rs = plan.factor(dev)
        torch.cuda.synchronize()
        for A, R in zip(As, Rs):
            assert _r_err(R.cpu().numpy(), A) <= 1e-11
        assert plan.info()["graph_captured"] == 1
    plan.close()


def test_batched_f32():
    import paper_0808_2664_amd as tq
    _note("case: batched f32")
    shapes = _shapes(40, 33, 64, 5000)
    As = [workloads.gaussian(m, n, 1500 + i).astype(np.float32) for i, (m, n) in enumerate(shapes)]
    plan = tq.BatchPlan(shapes, torch.float32)
    Rs = plan.factor([torch.from_numpy(a).cuda() for a in As])
    torch.cuda.synchronize()
    for A, R in zip(As, Rs):
        assert _r_err(R.double().cpu().numpy(), A.astype(np.float64)) <= 5e-4
    plan.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 5e-4)])
def test_config4_2000_matrices_sampled(dtype, tol):
    """The 2000-matrix batch (m ~ U{512..65536}, n in {8,16,32,64}, seed 6),
    one launch; sampled matrices checked against the oracle, every matrix
    checked through the column norms of R (equal to those of A)."""
    import paper_0808_2664_amd as tq
    from paper_0808_2664_amd import autotune
    _note("case: config4 batch of 2000, %s" % dtype)
    shapes = workloads.cfg4_shapes()
    As = [workloads.cfg4_device_matrix(i, m, n, dtype=dtype) for i, (m, n) in enumerate(shapes)]
    norms = [torch.linalg.vector_norm(A.double(), dim=0) for A in As]
    ms = np.array([m for m, _ in shapes])
    sample = sorted(set([0, 1, 999, 1999, int(ms.argmax()), int(ms.argmin())] +
                        [i for i, (m, n) in enumerate(shapes) if n == 64][:2]))
    keep = {i: As[i].double().cpu().numpy() for i in sample}
    plan = tq.BatchPlan(shapes, dtype, opts=autotune.choose_batch(shapes, dtype))
    Rs = plan.factor(As)
    torch.cuda.synchronize()
    worst = 0.0
    for i in sample:
        e = _r_err(Rs[i].double().cpu().numpy(), keep[i])
        worst = max(worst, e)
        assert e <= tol, (i, shapes[i], e)
    rel = max(float((torch.linalg.vector_norm(R.double(), dim=0) - nv).abs().max() / nv.max())
              for R, nv in zip(Rs, norms))
    _note("  worst sampled R error %.2e; worst column-norm mismatch %.2e" % (worst, rel))
    assert rel <= (1e-12 if dtype == torch.float64 else 1e-4)
    plan.close()
