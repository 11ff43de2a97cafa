"""GPU parity of the differentiable TSQR (QR adjoint kernels).

The oracle's adjoint is pinned on the CPU by central differences and a closed
form (tests/test_oracle.py); here the GPU gradients are compared with it and,
independently, with central differences of the GPU forward.
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


def test_adjoint_matches_oracle_and_fd_1024x8():
    import paper_0808_2664_amd as tq
    _note("case: adjoint 1024x8 f64")
    A = workloads.fd_case(1024, 8)
    rng = np.random.default_rng(12)
    dQ = rng.standard_normal(A.shape)
    dR = rng.standard_normal((8, 8))
    Ad = _dev(A).requires_grad_(True)
    Q, R = tq.tsqr(Ad)
    loss = (Q * _dev(dQ)).sum() + (R * _dev(dR)).sum()
    (g,) = torch.autograd.grad(loss, Ad)
    g = g.cpu().numpy()
    Qo, Ro = oracle.qr(A)
    go = oracle.qr_adjoint(Qo, Ro, dQ, dR)
    assert oracle.rel_err(g, go) <= 1e-11
    # central differences of the GPU forward (h = 1e-6)
    h = 1e-6
    scale = np.linalg.norm(go)
    for t in range(6):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        def f(X):
            Qx, Rx = tq.qr(_dev(X))
            return float((Qx.cpu().numpy() * dQ).sum() + (np.triu(Rx.cpu().numpy()) * dR).sum())
        fd = (f(A + h * E) - f(A - h * E)) / (2 * h)
        assert abs(fd - float((g * E).sum())) <= 1e-6 * scale


def test_adjoint_partial_upstream():
    import paper_0808_2664_amd as tq
    _note("case: adjoint with dQ only / dR only")
    A = workloads.gaussian(3000, 20, 21)
    Qo, Ro = oracle.qr(A)
    rng = np.random.default_rng(3)
    dQ = rng.standard_normal(A.shape)
    dR = rng.standard_normal((20, 20))
    Qd, Rd = _dev(Qo), _dev(Ro)
    gq = tq.qr_backward(Qd, Rd, _dev(dQ), None).cpu().numpy()
    gr = tq.qr_backward(Qd, Rd, None, _dev(dR)).cpu().numpy()
    assert oracle.rel_err(gq, oracle.qr_adjoint(Qo, Ro, dQ, np.zeros((20, 20)))) <= 1e-12
    assert oracle.rel_err(gr, oracle.qr_adjoint(Qo, Ro, np.zeros_like(dQ), dR)) <= 1e-12


@pytest.mark.parametrize("m,n", [(5000, 64), (777, 33), (100, 1)])
def test_adjoint_shapes(m, n):
    import paper_0808_2664_amd as tq
    _note("case: adjoint m=%d n=%d" % (m, n))
    A = workloads.gaussian(m, n, 40 + n)
    Qo, Ro = oracle.qr(A)
    rng = np.random.default_rng(n)
    dQ = rng.standard_normal(A.shape)
    dR = rng.standard_normal((n, n))
    g = tq.qr_backward(_dev(Qo), _dev(Ro), _dev(dQ), _dev(dR)).cpu().numpy()
    assert oracle.rel_err(g, oracle.qr_adjoint(Qo, Ro, dQ, dR)) <= 1e-12


def test_config5_fp64_262144x32():
    import paper_0808_2664_amd as tq
    _note("case: config5 fp64 262144x32")
    A, dQ, dR = workloads.cfg5()
    Ad = _dev(A).requires_grad_(True)
    Q, R = tq.tsqr(Ad)
    loss = (Q * _dev(dQ)).sum() + (R * _dev(dR)).sum()
    (g,) = torch.autograd.grad(loss, Ad)
    Qo, Ro = oracle.qr(A)
    go = oracle.qr_adjoint(Qo, Ro, dQ, dR)
    err = oracle.rel_err(g.cpu().numpy(), go)
    _note("  gradient error vs oracle %.2e" % err)
    assert err <= 1e-11


def test_config5_fp32_batch_all_members():
    """256 x 8192 x 32 FP32: the forward (one batched factorisation, every
    member on its own tree, then one explicit-Q pass) and the gradient of
    every member against the oracle on the rounded inputs."""
    import paper_0808_2664_amd as tq
    _note("case: config5 fp32 batch 256x8192x32 (all members)")
    A, dQ, dR = workloads.cfg5_batch()
    Ad = torch.from_numpy(A).cuda().requires_grad_(True)
    Q, R = tq.tsqr(Ad)
    loss = (Q * torch.from_numpy(dQ).cuda()).sum() + (R * torch.from_numpy(dR).cuda()).sum()
    (g,) = torch.autograd.grad(loss, Ad)
    g = g.double().cpu().numpy()
    Qg, Rg = Q.detach().double().cpu().numpy(), R.detach().double().cpu().numpy()
    worst = [0.0, 0.0, 0.0]
    for b in range(A.shape[0]):
        A64 = A[b].astype(np.float64)
        Qo, Ro = oracle.qr(A64)
        go = oracle.qr_adjoint(Qo, Ro, dQ[b].astype(np.float64), dR[b].astype(np.float64))
        worst[0] = max(worst[0], oracle.rel_err(Rg[b], Ro))
        worst[1] = max(worst[1], oracle.rel_err(Qg[b], Qo))
        worst[2] = max(worst[2], oracle.rel_err(g[b], go))
    _note("  worst member errors: R %.2e, Q %.2e, gradient %.2e" % tuple(worst))
    assert worst[0] <= 1e-5 and worst[1] <= 1e-5
    assert worst[2] <= 5e-4
