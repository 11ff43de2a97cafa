"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: values worked by hand
from the definition (tests/golden), 50-digit Gram-Schmidt on tiny inputs,
closed forms and special cases, library routines (Cholesky, lstsq), and the
invariants the paper's stability argument gives (Sec. 2.1: every step is an
orthogonal transformation).
"""
import json
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _frac(x):
    return float(Fraction(x))


def _fmat(rows):
    return np.array([[_frac(v) for v in r] for r in rows])


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- hand-worked

def test_hand_3x2_reflectors_and_R():
    g = _load("householder_3x2.json")
    A = _fmat(g["A"])
    YR, tau = oracle.geqrf(A)
    np.testing.assert_allclose(tau, [_frac(t) for t in g["tau"]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.r_of(YR), _fmat(g["R_raw"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(YR[1:, 0], [_frac(v) for v in g["v_tails"][0]], atol=1e-15)
    np.testing.assert_allclose(YR[2:, 1], [_frac(v) for v in g["v_tails"][1]], atol=1e-15)


def test_hand_3x2_q_and_apply():
    g = _load("householder_3x2.json")
    A = _fmat(g["A"])
    Q, R = oracle.qr(A)
    np.testing.assert_allclose(R, _fmat(g["R_normalised"]), atol=1e-15)
    np.testing.assert_allclose(Q, _fmat(g["Q_normalised"]), atol=1e-15)
    YR, tau = oracle.geqrf(A)
    b = np.array([_frac(v) for v in g["b"]])
    full = oracle.apply_qt(YR, tau, b)
    np.testing.assert_allclose(full, [_frac(v) for v in g["QT_b_full"]], atol=1e-15)
    d = oracle.signs(oracle.r_of(YR))
    thin = d * full[:2]
    np.testing.assert_allclose(thin, [_frac(v) for v in g["QT_b_thin_normalised"]], atol=1e-15)
    x = np.linalg.solve(R, thin)
    np.testing.assert_allclose(x, [_frac(v) for v in g["lstsq_x"]], atol=1e-15)
    assert abs(np.linalg.norm(full[2:]) - _frac(g["lstsq_residual_norm"])) < 1e-15


def test_hand_combine_4x2():
    g = _load("combine_4x2.json")
    # the leaves are already triangular: zero-tail branch, tau = 0, R unchanged
    for key in ("R0", "R1"):
        YR, tau = oracle.geqrf(_fmat(g[key]))
        assert np.all(tau == 0.0)
        np.testing.assert_array_equal(oracle.r_of(YR), _fmat(g[key]))
    S = _fmat(g["stacked"])
    YR, tau = oracle.geqrf(S)
    np.testing.assert_allclose(tau, [_frac(t) for t in g["tau"]], atol=1e-15)
    np.testing.assert_allclose(oracle.r_of(YR), _fmat(g["R_raw"]), atol=1e-15)
    V = np.zeros((4, 2))
    V[0, 0] = 1.0
    V[1:, 0] = YR[1:, 0]
    V[1, 1] = 1.0
    V[2:, 1] = YR[2:, 1]
    np.testing.assert_allclose(V.T, _fmat(g["v_full"]), atol=1e-15)
    # structure: the bottom-triangle part of the reflectors is upper triangular
    np.testing.assert_allclose(V[2:, :], _fmat(g["Y_bot"]), atol=1e-15)
    assert V[3, 0] == 0.0
    Q, R = oracle.qr(S)
    np.testing.assert_allclose(R, _fmat(g["R_normalised"]), atol=1e-14)


# ---------------------------------------------------------------- brute force

def _gs_decimal(A, digits=50):
    """Modified Gram-Schmidt in `digits`-digit decimal arithmetic."""
    getcontext().prec = digits
    m, n = A.shape
    cols = [[Decimal(repr(float(A[i, j]))) for i in range(m)] for j in range(n)]
    R = [[Decimal(0)] * n for _ in range(n)]
    Q = []
    for j in range(n):
        v = cols[j][:]
        for i in range(j):
            r = sum(Q[i][k] * v[k] for k in range(m))
            R[i][j] = r
            v = [v[k] - r * Q[i][k] for k in range(m)]
        # re-orthogonalise once (exact enough at 50 digits either way)
        for i in range(j):
            r = sum(Q[i][k] * v[k] for k in range(m))
            R[i][j] += r
            v = [v[k] - r * Q[i][k] for k in range(m)]
        nrm = sum(x * x for x in v).sqrt()
        R[j][j] = nrm
        Q.append([x / nrm for x in v])
    Qf = np.array([[float(Q[j][i]) for j in range(n)] for i in range(m)])
    Rf = np.array([[float(R[i][j]) for j in range(n)] for i in range(n)])
    return Qf, Rf


@pytest.mark.parametrize("m,n,seed", [(3, 2, 0), (4, 4, 1), (6, 3, 2), (8, 4, 3), (5, 1, 4), (7, 2, 5)])
def test_decimal_gram_schmidt(m, n, seed):
    A = workloads.gaussian(m, n, 100 + seed)
    Qx, Rx = _gs_decimal(A)
    Q, R = oracle.qr(A)
    assert oracle.rel_err(R, Rx) < 1e-15
    assert np.max(np.abs(Q - Qx)) < 1e-14


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("m,n", [(4096, 16), (3000, 64), (65, 64), (64, 64), (100, 1)])
def test_invariants_gaussian(m, n):
    A = workloads.gaussian(m, n, 7 + n)
    Q, R = oracle.qr(A)
    assert oracle.residual(A, Q, R) < 1e-13
    assert oracle.orthogonality(Q) < 1e-13
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(np.tril(R, -1), 0.0)
    # Cor. 1 (Sec. 4): R is the Cholesky factor of A^T A (well conditioned A)
    L = np.linalg.cholesky(A.T @ A)
    assert oracle.rel_err(R, L.T) < 1e-13


def test_invariants_ill_conditioned():
    A = workloads.conditioned(20000, 64, 1e8, 2, 3)
    Q, R = oracle.qr(A)
    assert oracle.residual(A, Q, R) < 1e-13
    assert oracle.orthogonality(Q) < 1e-13
    s = np.linalg.svd(R, compute_uv=False)
    assert 1e7 < s[0] / s[-1] < 1e9


def test_tau_range_and_unit_head():
    A = workloads.gaussian(300, 12, 21)
    YR, tau = oracle.geqrf(A)
    assert np.all((tau == 0) | ((tau >= 1.0) & (tau <= 2.0)))
    # H_j = I - tau v v^T must be orthogonal: tau = 2 / (v^T v) with v(0) = 1
    for j in range(12):
        v = np.concatenate([[1.0], YR[j + 1:, j]])
        assert abs(tau[j] * (v @ v) - 2.0) < 1e-14


# ---------------------------------------------------------------- special cases

def test_single_column_closed_form():
    a = workloads.gaussian(500, 1, 31)
    Q, R = oracle.qr(a)
    nrm = np.sqrt(np.sum(a[:, 0] ** 2))
    assert abs(R[0, 0] - nrm) < 1e-13 * nrm
    np.testing.assert_allclose(Q[:, 0], a[:, 0] / nrm, atol=1e-15)


def test_orthonormal_input_gives_identity():
    W = workloads.haar_orthogonal(40, 5)
    A = W[:, :16]
    Q, R = oracle.qr(A)
    np.testing.assert_allclose(R, np.eye(16), atol=1e-14)
    np.testing.assert_allclose(Q, A, atol=1e-14)


def test_triangle_over_zeros():
    rng = np.random.default_rng(9)
    R0 = np.triu(rng.standard_normal((10, 10)))
    A = np.vstack([R0, np.zeros((30, 10))])
    YR, tau = oracle.geqrf(A)
    assert np.all(tau == 0.0)
    Q, R = oracle.qr(A)
    d = oracle.signs(R0)
    np.testing.assert_allclose(R, d[:, None] * R0, atol=0)


def test_scaling_and_row_permutation():
    A = workloads.gaussian(900, 20, 41)
    Q, R = oracle.qr(A)
    Q2, R2 = oracle.qr(3.5 * A)
    assert oracle.rel_err(R2, 3.5 * R) < 1e-14
    assert oracle.rel_err(Q2, Q) < 1e-13
    # Sec. 2.2: rows in another order give the QR of a row permutation, same R
    perm = np.random.default_rng(4).permutation(900)
    Q3, R3 = oracle.qr(A[perm])
    assert oracle.rel_err(R3, R) < 1e-13
    assert oracle.rel_err(Q3, Q[perm]) < 1e-12


def test_zero_column_and_zero_block():
    A = workloads.gaussian(200, 8, 51)
    A[:, 3] = 0.0
    A[50:120, :] = 0.0
    YR, tau = oracle.geqrf(A)
    assert tau[3] == 0.0
    Q = oracle.form_q(YR, tau)
    R = oracle.r_of(YR)
    assert np.linalg.norm(A - Q @ R) / np.linalg.norm(A) < 1e-14
    assert oracle.orthogonality(Q) < 1e-14


# ---------------------------------------------------------------- apply / form

def test_apply_against_explicit_full_q():
    m, n, k = 60, 7, 5
    A = workloads.gaussian(m, n, 61)
    B = workloads.gaussian(m, k, 62)
    YR, tau = oracle.geqrf(A)
    Qfull = oracle.apply_q(YR, tau, np.eye(m))
    # Qfull is orthogonal, its first n columns are the thin Q, and Qfull^T A = [R; 0]
    np.testing.assert_allclose(Qfull.T @ Qfull, np.eye(m), atol=1e-14)
    np.testing.assert_allclose(Qfull[:, :n], oracle.form_q(YR, tau), atol=1e-15)
    RA = Qfull.T @ A
    np.testing.assert_allclose(RA[:n], oracle.r_of(YR), atol=1e-13)
    np.testing.assert_allclose(RA[n:], 0.0, atol=1e-13)
    np.testing.assert_allclose(oracle.apply_qt(YR, tau, B), Qfull.T @ B, atol=1e-14)
    np.testing.assert_allclose(oracle.apply_q(YR, tau, B), Qfull @ B, atol=1e-14)
    np.testing.assert_allclose(oracle.apply_q(YR, tau, oracle.apply_qt(YR, tau, B)), B, atol=1e-14)


def test_least_squares_matches_lstsq():
    m, n = 500, 9
    A = workloads.gaussian(m, n, 71)
    b = workloads.gaussian(m, 1, 72)[:, 0]
    YR, tau = oracle.geqrf(A)
    c = oracle.apply_qt(YR, tau, b)
    x = np.linalg.solve(oracle.r_of(YR), c[:n])
    xr, res, _, _ = np.linalg.lstsq(A, b, rcond=None)
    np.testing.assert_allclose(x, xr, rtol=1e-12, atol=1e-14)
    assert abs(np.sum(c[n:] ** 2) - res[0]) < 1e-10 * res[0]


def test_lstsq_hand_3x2():
    # x = (4/9, 1/9) and residual norm 1/3, worked by hand (golden fixture)
    g = _load("householder_3x2.json")
    A = _fmat(g["A"])
    b = np.array([_frac(v) for v in g["b"]])
    x, rn = oracle.lstsq(A, b)
    np.testing.assert_allclose(x, [_frac(v) for v in g["lstsq_x"]], rtol=0, atol=1e-15)
    assert abs(rn - _frac(g["lstsq_residual_norm"])) < 1e-15
    # two right-hand sides at once: b and 3b - A e_0 (solution 3x - e_0, residual 3 * 1/3)
    B = np.stack([b, 3 * b - A[:, 0]], axis=1)
    X, rns = oracle.lstsq(A, B)
    np.testing.assert_allclose(X[:, 0], x, atol=1e-15)
    np.testing.assert_allclose(X[:, 1], [3 * 4 / 9 - 1, 3 * 1 / 9], atol=1e-15)
    np.testing.assert_allclose(rns, [1 / 3, 1.0], atol=1e-15)


def test_lstsq_consistent_and_square_systems():
    # B = A X0 has the exact solution X0 and zero residual; a square A has no
    # residual rows at all
    A = workloads.gaussian(300, 12, 81)
    X0 = workloads.gaussian(12, 5, 82)
    X, rn = oracle.lstsq(A, A @ X0)
    np.testing.assert_allclose(X, X0, rtol=0, atol=1e-12)
    assert np.all(rn < 1e-12)
    S = workloads.gaussian(10, 10, 83) + 10 * np.eye(10)
    Bs = workloads.gaussian(10, 3, 84)
    Xs, rs = oracle.lstsq(S, Bs)
    np.testing.assert_allclose(Xs, np.linalg.solve(S, Bs), rtol=1e-12, atol=1e-13)
    assert np.all(rs == 0.0)


@pytest.mark.parametrize("m,n,k", [(500, 9, 4), (2000, 64, 3), (70, 64, 1)])
def test_lstsq_against_library_and_normal_equations(m, n, k):
    A = workloads.gaussian(m, n, 91 + n)
    B = workloads.gaussian(m, k, 92 + n)
    X, rn = oracle.lstsq(A, B)
    Xr, res, _, _ = np.linalg.lstsq(A, B, rcond=None)
    np.testing.assert_allclose(X, Xr, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(rn ** 2, res, rtol=1e-10)
    # the residual is orthogonal to range(A): A^T (A X - B) = 0
    Rs = A @ X - B
    assert np.linalg.norm(A.T @ Rs) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(Rs)
    np.testing.assert_allclose(np.linalg.norm(Rs, axis=0), rn, rtol=1e-12)


def test_cholqr_hand_3x2():
    # A^T A = [[9, 9], [9, 18]]: R = [[3, 3], [0, 3]], Q = A R^-1 (golden fixture)
    g = _load("householder_3x2.json")
    A = _fmat(g["A"])
    for passes in (1, 2):
        Q, R = oracle.cholqr(A, passes)
        np.testing.assert_allclose(R, _fmat(g["R_normalised"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(Q, _fmat(g["Q_normalised"]), rtol=0, atol=1e-15)


def test_cholqr_closed_form_u_times_triangle():
    # A = U T with orthonormal U and upper triangular T (positive diagonal):
    # A^T A = T^T T, so R = T and Q = U exactly (a transposed or mis-indexed
    # factor fails here)
    m, n = 400, 6
    U = np.linalg.qr(workloads.gaussian(m, n, 61))[0]
    T = np.triu(np.arange(1, n * n + 1, dtype=np.float64).reshape(n, n) % 7 + 1)
    for passes in (1, 2):
        Q, R = oracle.cholqr(U @ T, passes)
        np.testing.assert_allclose(R, T, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(Q, U, rtol=0, atol=1e-13)


def test_cholqr_matches_householder_r_and_loses_orthogonality():
    # R is unique with a positive diagonal (Sec. 4 Cor. 1: the Cholesky factor
    # of A^T A), so it matches the sign-normalised Householder R on a
    # well-conditioned input; at cond 1e7 one pass loses orthogonality
    # (~cond^2 u) and the second pass restores it
    A = workloads.gaussian(3000, 16, 62)
    Q, R = oracle.cholqr(A)
    Qh, Rh = oracle.qr(A)
    assert oracle.rel_err(R, Rh) < 1e-13
    assert oracle.orthogonality(Q) < 1e-13
    B = workloads.conditioned(3000, 16, 1e7, 63, 64)
    Q1, _ = oracle.cholqr(B, 1)
    Q2, R2 = oracle.cholqr(B, 2)
    assert oracle.orthogonality(Q1) > 1e-6
    assert oracle.orthogonality(Q2) < 1e-13
    assert oracle.residual(B, Q2, R2) < 1e-14
    with pytest.raises(FloatingPointError):
        oracle.cholqr(workloads.conditioned(3000, 16, 1e12, 65, 66))


def test_pairwise_sum():
    x = np.arange(1, 1001, dtype=np.float64)
    assert oracle.psum(x) == 500500.0
    # 1 + 2^-53 * many: sequential summation loses every small term,
    # the pairwise cascade keeps them once the small terms pair up
    y = np.full(1 << 12, 2.0 ** -53)
    y[0] = 1.0
    assert oracle.psum(y) > 1.0


# ---------------------------------------------------------------- adjoint

def _loss(A, dQ, dR):
    Q, R = oracle.qr(A)
    return float(np.sum(dQ * Q) + np.sum(np.triu(dR) * R))


def test_adjoint_central_fd():
    A = workloads.fd_case(1024, 8)
    rng = np.random.default_rng(12)
    dQ = rng.standard_normal(A.shape)
    dR = rng.standard_normal((8, 8))
    Q, R = oracle.qr(A)
    dA = oracle.qr_adjoint(Q, R, dQ, dR)
    h = 1e-6
    scale = np.linalg.norm(dA)
    for t in range(8):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (_loss(A + h * E, dQ, dR) - _loss(A - h * E, dQ, dR)) / (2 * h)
        assert abs(fd - np.sum(dA * E)) <= 1e-6 * scale


def test_adjoint_single_column_closed_form():
    a = workloads.gaussian(300, 1, 81)
    rng = np.random.default_rng(82)
    dq = rng.standard_normal((300, 1))
    dr = rng.standard_normal((1, 1))
    Q, R = oracle.qr(a)
    r = R[0, 0]
    q = Q[:, 0]
    # q = a/r, r = ||a||:  dA = (dq - q (q^T dq)) / r + q dr
    expect = (dq[:, 0] - q * (q @ dq[:, 0])) / r + q * dr[0, 0]
    dA = oracle.qr_adjoint(Q, R, dq, dr)
    np.testing.assert_allclose(dA[:, 0], expect, atol=1e-14)


def test_adjoint_ignores_lower_part_of_dR():
    A = workloads.gaussian(64, 5, 91)
    Q, R = oracle.qr(A)
    rng = np.random.default_rng(92)
    dQ = rng.standard_normal(A.shape)
    dR = rng.standard_normal((5, 5))
    a1 = oracle.qr_adjoint(Q, R, dQ, dR)
    a2 = oracle.qr_adjoint(Q, R, dQ, np.triu(dR))
    np.testing.assert_array_equal(a1, a2)


# ---------------------------------------------------------------- blocked Householder QR

@pytest.mark.parametrize("nb", [1, 2, 64])
def test_blocked_hand_3x2(nb):
    # panels of one or two columns: the compact form with T = tau (nb = 1) and
    # the 2 x 2 T of the whole matrix give the hand-worked reflectors and R
    g = _load("householder_3x2.json")
    YR, tau = oracle.geqrf_blocked(_fmat(g["A"]), nb)
    np.testing.assert_allclose(tau, [_frac(t) for t in g["tau"]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.r_of(YR), _fmat(g["R_raw"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(YR[1:, 0], [_frac(v) for v in g["v_tails"][0]], atol=1e-15)
    np.testing.assert_allclose(YR[2:, 1], [_frac(v) for v in g["v_tails"][1]], atol=1e-15)


def test_blocked_hand_combine_4x2():
    g = _load("combine_4x2.json")
    YR, tau = oracle.geqrf_blocked(_fmat(g["stacked"]), 1)
    np.testing.assert_allclose(tau, [_frac(t) for t in g["tau"]], atol=1e-15)
    np.testing.assert_allclose(oracle.r_of(YR), _fmat(g["R_raw"]), atol=1e-15)


@pytest.mark.parametrize("m,n,nb", [(300, 200, 16), (257, 130, 64), (1000, 700, 64), (5000, 96, 32),
                                    (64, 64, 64), (129, 128, 64), (2048, 2048, 64)])
def test_blocked_matches_unblocked(m, n, nb):
    # same reflectors, tau and R as the unblocked loop up to rounding: a
    # transposed T, a wrong recurrence sign or a skipped trailing column
    # fails here (n > nb in every case but one)
    A = workloads.gaussian(m, n, 70 + n)
    Y1, t1 = oracle.geqrf(A)
    Y2, t2 = oracle.geqrf_blocked(A, nb)
    assert oracle.rel_err(oracle.r_of(Y2), oracle.r_of(Y1)) < 1e-14
    np.testing.assert_allclose(t2, t1, rtol=0, atol=1e-12)
    L1, L2 = np.tril(Y1, -1), np.tril(Y2, -1)
    assert np.linalg.norm(L2 - L1) <= 1e-12 * np.linalg.norm(L1)


def test_blocked_invariants_and_thread_count():
    A = workloads.gaussian(1500, 1500, 77)
    Y, tau = oracle.geqrf_blocked(A, 64)
    Q = oracle.form_q(Y, tau)
    R = oracle.r_of(Y)
    assert oracle.residual(A, Q, R) < 1e-14
    assert oracle.orthogonality(Q) < 1e-12
    # R^T R = A^T A (Sec. 4 Cor. 1: R is the Cholesky factor of A^T A up to signs)
    assert np.linalg.norm(R.T @ R - A.T @ A) <= 1e-13 * np.linalg.norm(A) ** 2
    # every entry is computed by one thread in a fixed order
    nt = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        Y1, t1 = oracle.geqrf_blocked(A[:700, :600], 64)
        oracle.set_threads(max(2, nt))
        Y2, t2 = oracle.geqrf_blocked(A[:700, :600], 64)
    finally:
        oracle.set_threads(nt)
    np.testing.assert_array_equal(Y1, Y2)
    np.testing.assert_array_equal(t1, t2)


# ---------------------------------------------------------------- modified Gram-Schmidt

def test_mgs_hand_3x2():
    g = _load("householder_3x2.json")
    Q, R = oracle.mgs(_fmat(g["A"]))
    np.testing.assert_allclose(R, _fmat(g["R_normalised"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q, _fmat(g["Q_normalised"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("m,n,seed", [(3, 2, 0), (6, 3, 2), (8, 4, 3), (5, 1, 4)])
def test_mgs_decimal_gram_schmidt(m, n, seed):
    A = workloads.gaussian(m, n, 100 + seed)
    Qx, Rx = _gs_decimal(A)
    Q, R = oracle.mgs(A)
    assert oracle.rel_err(R, Rx) < 1e-15
    assert np.max(np.abs(Q - Qx)) < 1e-14


def test_mgs_closed_form_and_orthogonality_loss():
    # A = U T: R = T, Q = U
    m, n = 400, 6
    U = np.linalg.qr(workloads.gaussian(m, n, 81))[0]
    T = np.triu(np.arange(1, n * n + 1, dtype=np.float64).reshape(n, n) % 5 + 1)
    Q, R = oracle.mgs(U @ T)
    np.testing.assert_allclose(R, T, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(Q, U, rtol=0, atol=1e-13)
    # well conditioned: the Householder R; at cond 1e7 orthogonality is lost
    # in proportion to cond * u (MGS), not cond^2 * u (classical Gram-Schmidt
    # or CholeskyQR would exceed the upper bound)
    A = workloads.gaussian(3000, 16, 82)
    Q, R = oracle.mgs(A)
    assert oracle.rel_err(R, oracle.qr(A)[1]) < 1e-13
    assert oracle.orthogonality(Q) < 1e-13
    B = workloads.conditioned(3000, 16, 1e7, 83, 84)
    Qb, Rb = oracle.mgs(B)
    assert 1e-12 < oracle.orthogonality(Qb) < 1e-6
    assert oracle.residual(B, Qb, Rb) < 1e-14
    with pytest.raises(FloatingPointError):
        oracle.mgs(np.zeros((5, 2)))
