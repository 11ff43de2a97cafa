"""GPU parity of TSQR factor / apply_qt / apply_q / form_q against the oracle.

Gates (FP64, cond <= 1e8): normwise R error <= 1e-11; residual and
orthogonality <= 1e-13.  Q and the thin Q^T B are compared at 1e-11 for
well-conditioned inputs and at 100*cond*u otherwise (a property of the
problem, not of the algorithm: two correct QRs differ by ~cond*u there).
Rows n..m-1 of Q^T B depend on the tree; they are checked through their
column norms (the least-squares residual norms), which do not.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)


def _gram_pairwise(Q, chunk=1024):
    """Q^T Q with 1024-row chunks summed pairwise: a single GEMM over 2^20 rows
    has a summation error (~2e-13 on an exactly computed Q) larger than the
    1e-13 orthogonality gate, so the check itself must sum pairwise."""
    m, n = Q.shape
    pad = (-m) % chunk
    if pad:
        Q = torch.cat([Q, torch.zeros(pad, n, dtype=Q.dtype, device=Q.device)])
    Qc = Q.reshape(-1, chunk, n)
    G = torch.bmm(Qc.transpose(1, 2).contiguous(), Qc)
    while G.shape[0] > 1:
        if G.shape[0] % 2:
            G = torch.cat([G, torch.zeros_like(G[:1])])
        G = G[0::2] + G[1::2]
    return G[0]


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(A_np, B_np=None, dtype=torch.float64, **kw):
    import paper_0808_2664_amd as tq
    A = _dev(A_np, dtype)
    R, qt = tq.factor(A, **kw)
    Q = qt.form_q()
    out = {"R": R, "Q": Q, "qt": qt, "A": A}
    if B_np is not None:
        B = _dev(B_np, dtype)
        qt.apply_qt(B)
        out["QtB"] = B.clone()
        qt.apply_q(B)
        out["B_back"] = B
    torch.cuda.synchronize()
    return out


def _normalised(R, Q, QtB=None):
    R = R.double().cpu().numpy()
    d = oracle.signs(R)
    res = {"R": R * d[:, None], "Q": Q.double().cpu().numpy() * d[None, :]}
    if QtB is not None:
        X = QtB.double().cpu().numpy()
        res["thin"] = X[: R.shape[0]] * d[:, None]
        res["rest_norms"] = np.linalg.norm(X[R.shape[0]:], axis=0)
    return res


def _oracle(A, B=None):
    YR, tau = oracle.geqrf(A)
    R = oracle.r_of(YR)
    Q = oracle.form_q(YR, tau)
    d = oracle.signs(R)
    o = {"R": R * d[:, None], "Q": Q * d[None, :]}
    if B is not None:
        X = oracle.apply_qt(YR, tau, B)
        n = A.shape[1]
        o["thin"] = X[:n] * d[:, None]
        o["rest_norms"] = np.linalg.norm(X[n:], axis=0)
    return o


def _check(A, B, g, o, rtol_r=1e-11, rtol_q=1e-11, inv=1e-13):
    assert oracle.rel_err(g["R"], o["R"]) <= rtol_r
    assert oracle.rel_err(g["Q"], o["Q"]) <= rtol_q
    assert oracle.residual(A, g["Q"], g["R"]) <= inv
    assert oracle.orthogonality(g["Q"]) <= inv
    if B is not None:
        assert oracle.rel_err(g["thin"], o["thin"]) <= rtol_q
        np.testing.assert_allclose(g["rest_norms"], o["rest_norms"], rtol=max(rtol_q, 1e-12))


def test_config1_4096x16_f64():
    """4096 x 16, iid N(0,1) (seed 1), leaves of 256 rows, binary tree."""
    _note("case: config1 4096x16 f64")
    A = workloads.cfg1()
    B = workloads.gaussian(4096, 5, 99)
    out = _run(A, B, chains=16)
    info = out["qt"].info()
    assert info["chains"] == 16 and info["levels"] == 4 and info["arity"] == 2
    g = _normalised(out["R"], out["Q"], out["QtB"])
    _check(A, B, g, _oracle(A, B))
    np.testing.assert_allclose(out["B_back"].cpu().numpy(), B, atol=1e-13)


SHAPES = [
    # m, n, block_rows, chains, arity
    (64, 64, 64, 0, 0),
    (100, 1, 64, 0, 0),
    (1000, 3, 64, 0, 0),
    (1000, 8, 64, 5, 3),
    (777, 31, 64, 0, 0),
    (2049, 32, 64, 0, 0),
    (2500, 33, 64, 3, 2),
    (5000, 64, 64, 0, 0),
    (5000, 64, 64, 1, 0),
    (3333, 64, 64, 7, 4),
    (20000, 16, 64, 10, 2),
    (300, 64, 64, 2, 3),
    (129, 64, 64, 0, 0),
    (4100, 20, 64, 0, 2),
    (70000, 64, 64, 0, 2),
    (100000, 48, 64, 0, 3),
    (3000, 12, 64, 0, 0),
    (9999, 5, 64, 0, 7),
    (262144 + 3, 17, 64, 0, 2),
]


@pytest.mark.parametrize("m,n,h,chains,arity", SHAPES)
def test_shapes_f64(m, n, h, chains, arity):
    _note("case: shape m=%d n=%d h=%d chains=%d arity=%d" % (m, n, h, chains, arity))
    A = workloads.gaussian(m, n, 1000 + m + n)
    B = workloads.gaussian(m, 17, 2000 + m)
    out = _run(A, B, block_rows=h, chains=chains, arity=arity)
    g = _normalised(out["R"], out["Q"], out["QtB"])
    _check(A, B, g, _oracle(A, B))
    np.testing.assert_allclose(out["B_back"].cpu().numpy(), B, atol=1e-12)


def test_zero_column_and_zero_block():
    _note("case: zero column / zero block")
    A = workloads.gaussian(3000, 16, 77)
    A[:, 5] = 0.0
    A[700:1500, :] = 0.0
    out = _run(A, None, chains=5)
    R = out["R"].cpu().numpy()
    Q = out["Q"].cpu().numpy()
    assert abs(R[5, 5]) == 0.0
    assert oracle.residual(A, Q, R) <= 1e-13
    assert oracle.orthogonality(Q) <= 1e-13


def test_triangular_input_zero_tails():
    _note("case: triangle over zeros")
    rng = np.random.default_rng(5)
    R0 = np.triu(rng.standard_normal((16, 16)))
    A = np.vstack([R0, np.zeros((1000, 16))])
    out = _run(A, None, block_rows=64)
    g = _normalised(out["R"], out["Q"])
    d = oracle.signs(R0)
    np.testing.assert_allclose(g["R"], R0 * d[:, None], atol=1e-14)


def test_hand_worked_combine_node():
    """The 4x2 tree node of tests/golden/combine_4x2.json, embedded as two
    64-row chains whose leaves are the given triangles over zeros."""
    import json
    import os
    from fractions import Fraction
    _note("case: golden combine node")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "combine_4x2.json")))
    f = lambda rows: np.array([[float(Fraction(v)) for v in r] for r in rows])
    A = np.zeros((128, 2))
    A[0:2] = f(g["R0"])
    A[64:66] = f(g["R1"])
    out = _run(A, None, block_rows=64, chains=2)
    np.testing.assert_allclose(out["R"].cpu().numpy(), f(g["R_raw"]), atol=1e-14)


def test_determinism_bitwise():
    _note("case: determinism")
    A = workloads.gaussian(50000, 64, 3)
    Rs = []
    for _ in range(3):
        out = _run(A, None)
        Rs.append(out["R"].cpu().numpy())
    assert np.array_equal(Rs[0], Rs[1]) and np.array_equal(Rs[0], Rs[2])


def test_tree_shape_invariance():
    """Sec. 2.1: any reduction tree gives the same R up to roundoff and signs."""
    _note("case: tree shapes")
    A = workloads.gaussian(40000, 32, 8)
    Rs = []
    for kw in [dict(), dict(chains=1), dict(chains=9, arity=3), dict(chains=625, arity=2), dict(chains=40, arity=5)]:
        out = _run(A, None, **kw)
        Rs.append(_normalised(out["R"], out["Q"])["R"])
    for R in Rs[1:]:
        assert oracle.rel_err(R, Rs[0]) <= 1e-13


@pytest.mark.parametrize("m,n,chains,dt", [
    (1 << 16, 64, 0, "f64"),      # 1024 chains of one block, 10 levels
    (100000, 48, 37, "f64"),      # W not a power of two: unpaired positions
    (70000, 17, 300, "f64"),      # two panels, the second with one live column
    (50000, 8, 200, "f64"),       # one panel
    (40000, 64, 3, "f64"),        # two levels, an unpaired chain at the top
    (1 << 16, 64, 513, "f32"),
    (150000, 8, 2000, "f64"),     # 2000 waves, two per SIMD, still all resident
    (200000, 64, 2000, "f64"),    # more chains than resident waves: node-by-node fallback
])
def test_pipelined_tree_matches_levelwise(m, n, chains, dt):
    """The panel-pipelined tree and the node-by-node tree perform the same
    node arithmetic in the same order: R, the reflectors and Q agree bitwise,
    and R matches the oracle."""
    import paper_0808_2664_amd as tq
    _note("case: pipelined vs levelwise tree m=%d n=%d chains=%d %s" % (m, n, chains, dt))
    dtype = torch.float64 if dt == "f64" else torch.float32
    A_np = workloads.gaussian(m, n, 21)
    outs = []
    for lw in (False, True):
        A = _dev(A_np, dtype)
        R, qt = tq.factor(A, chains=chains, levelwise=lw)
        Q = qt.form_q()
        torch.cuda.synchronize()
        outs.append((R.clone(), A.clone(), Q))
        qt.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])
    g = _normalised(outs[0][0], outs[0][2])
    o = _oracle(A_np, None)
    assert oracle.rel_err(g["R"], o["R"]) <= (1e-11 if dt == "f64" else 5e-4)


def test_f32_gaussian():
    _note("case: f32")
    A = workloads.gaussian(30000, 32, 12).astype(np.float32)
    B = workloads.gaussian(30000, 4, 13).astype(np.float32)
    out = _run(A, B, dtype=torch.float32)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    g = _normalised(out["R"], out["Q"], out["QtB"])
    o = _oracle(A64, B64)
    assert oracle.rel_err(g["R"], o["R"]) <= 5e-4
    assert oracle.residual(A64, g["Q"], g["R"]) <= 1e-5
    assert oracle.orthogonality(g["Q"]) <= 1e-4
    assert oracle.rel_err(g["thin"], o["thin"]) <= 5e-4


def test_ill_conditioned_1e8():
    _note("case: cond 1e8 (2^16 x 64)")
    A = workloads.conditioned(1 << 16, 64, 1e8, 2, 3)
    B = workloads.gaussian(1 << 16, 32, 4)
    out = _run(A, B)
    g = _normalised(out["R"], out["Q"], out["QtB"])
    o = _oracle(A, B)
    tol_q = 100 * 1e8 * U64
    _check(A, B, g, o, rtol_r=1e-11, rtol_q=tol_q)


def test_config2_full_size_against_oracle():
    """2^20 x 64, cond 1e8, B 2^20 x 32: the configuration the bench times, in
    the bench's launch configuration (1024 chains of 16 blocks, pipelined
    tree, wide apply kernels).  The whole R, the whole thin Q and the whole
    thin Q^T B against the oracle's Householder QR (the oracle's form_q and
    apply_qt on its own reflectors); R is also pinned by its leading block
    (the R of A[:, :16]) and its column norms; residual and orthogonality."""
    _note("case: config2 full size")
    A, B = workloads.cfg2()
    YRo, tauo = oracle.geqrf(A)
    Ro_full = oracle.r_of(YRo)
    do = oracle.signs(Ro_full)
    import paper_0808_2664_amd as tq
    Ad = _dev(A)
    R, qt = tq.factor(Ad)
    info = qt.info()
    assert info["chains"] == 1024 and info["blocks"] == 16384
    assert qt.wide_layout(32) and qt.wide_layout(64)
    Q = qt.form_q()
    Bd = _dev(B)
    qt.apply_qt(Bd)
    torch.cuda.synchronize()
    Rn = R.cpu().numpy()
    d = oracle.signs(Rn)
    Rn = Rn * d[:, None]
    k = 16
    YRk, tauk = oracle.geqrf(A[:, :k])
    Rk = oracle.r_of(YRk)
    dk = oracle.signs(Rk)
    assert oracle.rel_err(Rn[:k, :k], Rk * dk[:, None]) <= 1e-11
    np.testing.assert_allclose(np.linalg.norm(Rn, axis=0), np.linalg.norm(A, axis=0), rtol=1e-12)
    assert oracle.rel_err(Rn, Ro_full * do[:, None]) <= 1e-11
    # thin Q and thin Q^T B against the oracle: at cond 1e8 two correct QRs
    # differ by about cond * u in these, so the gate is 100 cond u
    gate = 100 * 1e8 * U64
    Qo = oracle.form_q(YRo, tauo) * do[None, :]
    Qn = Q.cpu().numpy() * d[None, :]
    eq = oracle.rel_err(Qn, Qo)
    thin_o = oracle.apply_qt(YRo, tauo, B)[:64] * do[:, None]
    thin = Bd[:64].cpu().numpy() * d[:, None]
    eb = oracle.rel_err(thin, thin_o)
    _note("  Q error %.2e, thin Q^T B error %.2e (gate %.1e)" % (eq, eb, gate))
    assert eq <= gate and eb <= gate
    # the trailing rows of Q^T B depend on the tree; their column norms do not
    tail_o = np.linalg.norm(oracle.apply_qt(YRo, tauo, B)[64:], axis=0)
    tail = torch.linalg.norm(Bd[64:], dim=0).cpu().numpy()
    np.testing.assert_allclose(tail, tail_o, rtol=1e-11)
    Qd = Q * _dev(d)[None, :]
    Rd = _dev(Rn)
    res = (torch.linalg.norm(_dev(A) - Qd @ Rd) / torch.linalg.norm(_dev(A))).item()
    orth = torch.linalg.norm(_gram_pairwise(Qd) - torch.eye(64, dtype=torch.float64, device="cuda")).item()
    assert res <= 1e-13 and orth <= 1e-13
    qt.close()


@pytest.mark.parametrize("k", [32, 64])
def test_f32_wide_apply_against_oracle(k):
    """FP32 storage and compute with the wide apply kernels (2^16 x 64, 1024
    chains): Q^T B, Q B and the explicit Q against the oracle run in FP64 on
    the rounded inputs."""
    _note("case: f32 wide apply k=%d" % k)
    m, n = 1 << 16, 64
    A = workloads.gaussian(m, n, 910).astype(np.float32)
    B = workloads.gaussian(m, k, 911).astype(np.float32)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    import paper_0808_2664_amd as tq
    Ad = _dev(A, torch.float32)
    R, qt = tq.factor(Ad)
    assert qt.wide_layout(k)
    Q = qt.form_q()
    Bd = _dev(B, torch.float32)
    qt.apply_qt(Bd)
    thin = Bd[:n].double().cpu().numpy()
    tail = torch.linalg.norm(Bd[n:].double(), dim=0).cpu().numpy()
    qt.apply_q(Bd)
    back = Bd.double().cpu().numpy()
    torch.cuda.synchronize()
    YRo, tauo = oracle.geqrf(A64)
    Ro = oracle.r_of(YRo)
    do = oracle.signs(Ro)
    Rg = R.double().cpu().numpy()
    d = oracle.signs(Rg)
    assert oracle.rel_err(Rg * d[:, None], Ro * do[:, None]) <= 1e-5
    assert oracle.rel_err(Q.double().cpu().numpy() * d[None, :], oracle.form_q(YRo, tauo) * do[None, :]) <= 1e-5
    full_o = oracle.apply_qt(YRo, tauo, B64)
    assert oracle.rel_err(thin * d[:, None], full_o[:n] * do[:, None]) <= 1e-5
    np.testing.assert_allclose(tail, np.linalg.norm(full_o[n:], axis=0), rtol=1e-5)
    assert oracle.rel_err(back, B64) <= 1e-5  # Q (Q^T B) = B
    qt.close()


def test_apply_qt_and_form_q_concurrent_streams():
    """apply_qt and form_q on two streams at once (the benchmark's schedule)
    give the same bits as one after the other, on 2^18 x 64 FP64 with 256
    chains (wide apply kernels, tree kernels by last arrival), and Q^T B
    matches the oracle's column norms."""
    import paper_0808_2664_amd as tq
    _note("case: apply_qt || form_q on two streams, 262144 x 64")
    m, n, k = 1 << 18, 64, 32
    A = workloads.gaussian(m, n, 920)
    B = workloads.gaussian(m, k, 921)
    Ad = _dev(A)
    R, qt = tq.factor(Ad, chains=256)
    B1, B2 = _dev(B), _dev(B)
    Q1 = torch.empty(m, n, dtype=torch.float64, device="cuda")
    Q2 = torch.empty_like(Q1)
    qt.apply_qt(B1)
    qt.form_q(Q1)
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    for _ in range(3):
        side.wait_stream(main)
        with torch.cuda.stream(side):
            qt.apply_qt(B2)
        qt.form_q(Q2)
        main.wait_stream(side)
        torch.cuda.synchronize()
        assert torch.equal(Q1, Q2)
        assert torch.equal(B1, B2)
        B2.copy_(_dev(B))
    torch.cuda.synchronize()
    qt.close()
    YRo, tauo = oracle.geqrf(A)
    np.testing.assert_allclose(np.linalg.norm(B1[:n].cpu().numpy(), axis=0),
                               np.linalg.norm(oracle.apply_qt(YRo, tauo, B)[:n], axis=0), rtol=1e-12)


@pytest.mark.parametrize("m,n,chains,dt", [(1 << 20, 64, 0, "f64"), (300000, 32, 1024, "f32")])
def test_pipelined_tree_beside_concurrent_work(m, n, chains, dt):
    """The panel-pipelined tree is an ordinary launch whose waves all fit on
    the device.  With another stream keeping the device busy (large FP32
    matmuls issued first), workgroups of the tree that cannot start at once
    start as that work retires, so every wait ends: the same bits as a run on
    an idle device, and no bounded wait gave up."""
    import paper_0808_2664_amd as tq
    _note("case: pipelined tree beside concurrent work m=%d n=%d %s" % (m, n, dt))
    dtype = torch.float64 if dt == "f64" else torch.float32
    A_np = workloads.gaussian(m, n, 31)
    A = _dev(A_np, dtype)
    R0, qt = tq.factor(A, chains=chains)
    Q0 = qt.form_q()
    torch.cuda.synchronize()
    qt.close()
    assert tq.check_status() == 0
    X = torch.randn(8192, 8192, device="cuda")
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    for _ in range(2):
        A = _dev(A_np, dtype)
        side.wait_stream(main)
        with torch.cuda.stream(side):
            Y = X
            for _ in range(6):
                Y = torch.mm(Y, X) * 1e-3
        R, qt = tq.factor(A, chains=chains)
        Q = qt.form_q()
        main.wait_stream(side)
        torch.cuda.synchronize()
        qt.close()
        assert tq.check_status() == 0
        assert torch.equal(R, R0) and torch.equal(Q, Q0)
