/*
 * CPU FP64 oracle for the QR path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU product path shares no code with it.
 *
 * What it computes: the thin QR factorisation A = QR of an m x n matrix,
 * m >= n, by conventional Householder reduction.  In the paper's terms this
 * is the "trivial tree" (one reduction node holding every row), which the
 * paper states is conventional Householder QR (Sec. 2.1, the trivial-tree
 * picture following Eq. TSQR_binarytree_4).  Every TSQR tree and CAQR reach
 * the same factorisation in exact arithmetic, up to the signs of diag(R)
 * (Sec. 2.1, uniqueness remark after Eq. TSQR_binarytree_4), so this is the
 * plain definition the GPU path is compared against.
 *
 * Conventions (readings of the paper, see the design notes):
 *  - Householder vectors have unit topmost nonzero entry, H = I - tau v v^T
 *    (Sec. 5.2, the normalisation used for the dependency argument).
 *  - beta = -sign(alpha) * ||x||, with sign(0) = +1; tau = 0 (no reflection)
 *    when the tail below the diagonal is exactly zero.
 *  - Every reduction over rows uses pairwise summation.
 *
 * Storage: the public entry points take row-major, contiguous arrays (C order,
 * as numpy stores them).  Internally the factorisation works on a
 * column-major copy so that columns are contiguous.
 *
 * Functions without an independent pin are marked "parity unpinned" in their
 * comment; at present every exported function is pinned by the CPU tests.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Pairwise (cascade) summation of x[0..n): split in halves down to blocks of
 * at most 8 terms which are summed left to right. */
static double psum(const double *x, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += x[i];
        return s;
    }
    int64_t h = n / 2;
    return psum(x, h) + psum(x + h, n - h);
}

/* Scratch buffer for products fed to psum. */
typedef struct {
    double *p;
    int64_t cap;
} scratch_t;

static int scratch_reserve(scratch_t *s, int64_t n)
{
    if (n <= s->cap)
        return 0;
    free(s->p);
    s->p = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    s->cap = s->p ? n : 0;
    return s->p ? 0 : -1;
}

/* sum_i a[i]*b[i] with pairwise summation of the products */
static double pdot(scratch_t *s, const double *a, const double *b, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        s->p[i] = a[i] * b[i];
    return psum(s->p, n);
}

/* Householder QR of a column-major m x n matrix (leading dimension m).
 * On exit: R on and above the diagonal, v(1:) below it (v(0) = 1 implicit),
 * tau[j] per column.  Returns 0, or -1 on allocation failure.
 * The updates of the columns k > j are independent of one another and are
 * shared among OpenMP threads; each column's arithmetic is the same whatever
 * the thread count, so the result does not depend on it. */
static int geqr2_cm(int64_t m, int64_t n, double *a, double *tau)
{
    scratch_t s = {0, 0};
    if (scratch_reserve(&s, m) != 0)
        return -1;
    int fail = 0;
    for (int64_t j = 0; j < n && j < m; ++j) {
        double *x = a + j * m + j; /* column j, rows j..m-1 */
        int64_t len = m - j;
        double alpha = x[0];
        double sigma2 = (len > 1) ? pdot(&s, x + 1, x + 1, len - 1) : 0.0;
        if (sigma2 == 0.0) {
            /* no reflection: H_j = I, R_jj = alpha, tail already zero */
            tau[j] = 0.0;
        } else {
            double nrm = hypot(alpha, sqrt(sigma2));
            double beta = (alpha >= 0.0) ? -nrm : nrm; /* sign(0) = +1 */
            tau[j] = (beta - alpha) / beta;
            double scale = 1.0 / (alpha - beta);
            for (int64_t i = 1; i < len; ++i)
                x[i] *= scale;
            x[0] = beta;
        }
        if (tau[j] == 0.0)
            continue;
        /* apply H_j = I - tau v v^T to columns k > j, rows j..m-1 */
        const double tj = tau[j];
#pragma omp parallel if ((n - j - 1) * len > 65536)
        {
            scratch_t ts = {0, 0};
            int ok = scratch_reserve(&ts, len) == 0;
            if (!ok) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(static)
            for (int64_t k = j + 1; k < n; ++k) {
                if (!ok)
                    continue;
                double *c = a + k * m + j;
                /* w = v^T c with v(0) = 1 */
                ts.p[0] = c[0];
                for (int64_t i = 1; i < len; ++i)
                    ts.p[i] = x[i] * c[i];
                double w = psum(ts.p, len);
                double tw = tj * w;
                c[0] -= tw;
                for (int64_t i = 1; i < len; ++i)
                    c[i] -= tw * x[i];
            }
            free(ts.p);
        }
        if (fail)
            break;
    }
    free(s.p);
    return fail ? -1 : 0;
}

static double *to_cm(int64_t m, int64_t n, const double *rm)
{
    double *cm = (double *)malloc((size_t)(m * n > 0 ? m * n : 1) * sizeof(double));
    if (!cm)
        return NULL;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            cm[j * m + i] = rm[i * n + j];
    return cm;
}

static void from_cm(int64_t m, int64_t n, const double *cm, double *rm)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            rm[i * n + j] = cm[j * m + i];
}

/* Householder QR, row-major in place (LAPACK xGEQR2 output layout).
 * A: m x n row-major.  On exit R is in the upper triangle and the reflector
 * tails v(1:) are below the diagonal.  tau: n entries.
 * Returns 0, -1 for bad sizes, -2 on allocation failure. */
int oracle_geqrf(int64_t m, int64_t n, double *A, double *tau)
{
    if (m < 0 || n < 0 || m < n)
        return -1;
    double *cm = to_cm(m, n, A);
    if (!cm)
        return -2;
    int rc = geqr2_cm(m, n, cm, tau);
    from_cm(m, n, cm, A);
    free(cm);
    return rc == 0 ? 0 : -2;
}

/* Apply H_j = I - tau_j v_j v_j^T for j in order (first..last step dir) to the
 * m x k row-major B, where v_j comes from the geqrf output YR (m x n).  The
 * k columns of B are independent and are shared among OpenMP threads; each
 * column's arithmetic is the same whatever the thread count. */
static int apply_reflectors(int64_t m, int64_t n, int64_t k, const double *YR,
                            const double *tau, double *B, int forward)
{
    if (m < 0 || n < 0 || k < 0 || m < n)
        return -1;
    double *bc = to_cm(m, k, B);
    double *yc = to_cm(m, n, YR);
    if (!bc || !yc) {
        free(bc);
        free(yc);
        return -2;
    }
    int fail = 0;
#pragma omp parallel if (k > 1 && m * n > 65536)
    {
        scratch_t s = {0, 0};
        int ok = scratch_reserve(&s, m) == 0;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(static)
        for (int64_t c = 0; c < k; ++c) {
            if (!ok)
                continue;
            for (int64_t step = 0; step < n; ++step) {
                int64_t j = forward ? step : n - 1 - step;
                if (tau[j] == 0.0)
                    continue;
                const double *v = yc + j * m + j; /* v(0)=1 implicit, v(1:) stored */
                int64_t len = m - j;
                double *b = bc + c * m + j;
                s.p[0] = b[0];
                for (int64_t i = 1; i < len; ++i)
                    s.p[i] = v[i] * b[i];
                double tw = tau[j] * psum(s.p, len);
                b[0] -= tw;
                for (int64_t i = 1; i < len; ++i)
                    b[i] -= tw * v[i];
            }
        }
        free(s.p);
    }
    if (!fail)
        from_cm(m, k, bc, B);
    free(bc);
    free(yc);
    return fail ? -2 : 0;
}

/* B (m x k) <- Q^T B, Q = H_0 H_1 ... H_{n-1} (so Q^T applies H_0 first). */
int oracle_apply_qt(int64_t m, int64_t n, int64_t k, const double *YR,
                    const double *tau, double *B)
{
    return apply_reflectors(m, n, k, YR, tau, B, 1);
}

/* B (m x k) <- Q B (H_{n-1} first). */
int oracle_apply_q(int64_t m, int64_t n, int64_t k, const double *YR,
                   const double *tau, double *B)
{
    return apply_reflectors(m, n, k, YR, tau, B, 0);
}

/* Thin Q (m x n, row-major) = Q [I_n; 0]. */
int oracle_form_q(int64_t m, int64_t n, const double *YR, const double *tau,
                  double *Q)
{
    if (m < 0 || n < 0 || m < n)
        return -1;
    memset(Q, 0, (size_t)(m * n) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        Q[i * n + i] = 1.0;
    return apply_reflectors(m, n, n, YR, tau, Q, 0);
}

/*
 * Adjoint (reverse-mode derivative) of the thin QR map A -> (Q, R) with the
 * normalisation diag(R) > 0.  Not in the paper; this is the published QR
 * adjoint (Walter & Lehmann; the "copyltu" form of Liao, Liu, Wang & Xiang):
 *     M    = R * triu(dR)^T - dQ^T * Q                     (n x n)
 *     C    = tril(M) + tril(M, -1)^T                       (copyltu)
 *     dA   = (dQ + Q * C) * R^{-T}
 * Inputs (row-major): Q m x n, R n x n (upper, positive diagonal), dQ m x n,
 * dR n x n (only its upper triangle is used).  Output dA m x n.
 * Sums over the m rows are pairwise; the triangular solve is plain
 * substitution, row by row.
 */
int oracle_qr_adjoint(int64_t m, int64_t n, const double *Q, const double *R,
                      const double *dQ, const double *dR, double *dA)
{
    if (m < 0 || n < 0 || m < n)
        return -1;
    double *Mx = (double *)calloc((size_t)(n * n > 0 ? n * n : 1), sizeof(double));
    double *qc = to_cm(m, n, Q);
    double *dqc = to_cm(m, n, dQ);
    scratch_t s = {0, 0};
    if (!Mx || !qc || !dqc || scratch_reserve(&s, m > n ? m : n) != 0) {
        free(Mx);
        free(qc);
        free(dqc);
        free(s.p);
        return -2;
    }
    /* M = R triu(dR)^T - dQ^T Q */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            /* (R triu(dR)^T)_{ij} = sum_l R[i][l] * triu(dR)[j][l] */
            for (int64_t l = 0; l < n; ++l) {
                double r = (l >= i) ? R[i * n + l] : 0.0;
                double d = (l >= j) ? dR[j * n + l] : 0.0;
                acc += r * d;
            }
            double g = pdot(&s, dqc + i * m, qc + j * m, m);
            Mx[i * n + j] = acc - g;
        }
    }
    /* C = copyltu(M): lower triangle kept, mirrored to the upper one */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            Mx[i * n + j] = Mx[j * n + i];
    /* Bm = dQ + Q C ; then dA = Bm R^{-T}, i.e. each row x solves R x^T = b^T */
    double *b = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!b) {
        free(Mx);
        free(qc);
        free(dqc);
        free(s.p);
        return -2;
    }
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t j = 0; j < n; ++j) {
            double acc = dQ[r * n + j];
            for (int64_t l = 0; l < n; ++l)
                acc += Q[r * n + l] * Mx[l * n + j];
            b[j] = acc;
        }
        /* back substitution: R x = b, R upper triangular */
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = b[i];
            for (int64_t l = i + 1; l < n; ++l)
                acc -= R[i * n + l] * dA[r * n + l];
            dA[r * n + i] = acc / R[i * n + i];
        }
    }
    free(b);
    free(Mx);
    free(qc);
    free(dqc);
    free(s.p);
    return 0;
}

/*
 * Linear least squares: for each column b of B (m x k), the x minimising
 * ||A x - b||_2, A m x n of full column rank (m >= n).  The QR factorisation
 * is the paper's tool for this problem (Sec. 1, the remark on solving a least
 * squares problem with TSQR): with A = Q R and c = Q^T b (full m x m Q),
 * x solves R x = c(0:n) and the residual norm is ||c(n:m)||_2, since Q
 * preserves norms.  Steps: Householder QR (oracle_geqrf), Q^T B
 * (oracle_apply_qt), back substitution row by row from the last, and a
 * pairwise sum of the squares of the trailing m - n entries per column.
 * Inputs row-major: A m x n, B m x k.  Outputs: X n x k (row-major), rnorm
 * k entries.  Returns 0, -1 for bad sizes, -2 on allocation failure.
 */
int oracle_lstsq(int64_t m, int64_t n, int64_t k, const double *A, const double *B,
                 double *X, double *rnorm)
{
    if (m < 0 || n < 0 || k < 0 || m < n)
        return -1;
    double *yr = (double *)malloc((size_t)(m * n > 0 ? m * n : 1) * sizeof(double));
    double *tau = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *c = (double *)malloc((size_t)(m * k > 0 ? m * k : 1) * sizeof(double));
    double *sq = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!yr || !tau || !c || !sq) {
        free(yr);
        free(tau);
        free(c);
        free(sq);
        return -2;
    }
    memcpy(yr, A, (size_t)(m * n) * sizeof(double));
    memcpy(c, B, (size_t)(m * k) * sizeof(double));
    int rc = oracle_geqrf(m, n, yr, tau);
    if (rc == 0)
        rc = oracle_apply_qt(m, n, k, yr, tau, c);
    if (rc != 0) {
        free(yr);
        free(tau);
        free(c);
        free(sq);
        return rc == -1 ? -1 : -2;
    }
    for (int64_t col = 0; col < k; ++col) {
        /* R x = c(0:n): R is the upper triangle of yr */
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = c[i * k + col];
            for (int64_t l = i + 1; l < n; ++l)
                acc -= yr[i * n + l] * X[l * k + col];
            X[i * k + col] = acc / yr[i * n + i];
        }
        for (int64_t i = n; i < m; ++i)
            sq[i - n] = c[i * k + col] * c[i * k + col];
        rnorm[col] = sqrt(psum(sq, m - n));
    }
    free(yr);
    free(tau);
    free(c);
    free(sq);
    return 0;
}

/*
 * CholeskyQR, the fast but conditionally stable alternative the paper
 * compares TSQR with (Sec. 2.3 and its sequential cost table): G = A^T A,
 * R = the upper triangular Cholesky factor of G (R^T R = G, positive
 * diagonal), Q = A R^{-1}.  With passes = 2 (CholeskyQR2) the same steps are
 * applied to Q, giving Q2 and R2, and R = R2 R1.
 * Textbook steps: G entries by pairwise sums over the m rows; Cholesky
 * R_jj = sqrt(G_jj - sum_{k<j} R_kj^2), R_jc = (G_jc - sum_{k<j} R_kj R_kc) / R_jj;
 * each row q of Q from q R = a by forward substitution.
 * Inputs row-major: A m x n.  Outputs: Q m x n, R n x n (zeros below the
 * diagonal).  Returns 0, -1 for bad sizes, -2 on allocation failure, -3 if a
 * Cholesky pivot is not positive (G not numerically positive definite).
 */
static int cholqr_pass(int64_t m, int64_t n, const double *A, double *Q, double *R)
{
    double *ac = to_cm(m, n, A);
    scratch_t s = {0, 0};
    double *G = (double *)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(double));
    if (!ac || !G || scratch_reserve(&s, m > 0 ? m : 1) != 0) {
        free(ac);
        free(G);
        free(s.p);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j)
            G[i * n + j] = pdot(&s, ac + i * m, ac + j * m, m);
    free(ac);
    free(s.p);
    int rc = 0;
    memset(R, 0, (size_t)(n * n) * sizeof(double));
    for (int64_t j = 0; j < n && rc == 0; ++j) {
        double d = G[j * n + j];
        for (int64_t k = 0; k < j; ++k)
            d -= R[k * n + j] * R[k * n + j];
        if (!(d > 0.0)) {
            rc = -3;
            break;
        }
        R[j * n + j] = sqrt(d);
        for (int64_t c = j + 1; c < n; ++c) {
            double v = G[j * n + c];
            for (int64_t k = 0; k < j; ++k)
                v -= R[k * n + j] * R[k * n + c];
            R[j * n + c] = v / R[j * n + j];
        }
    }
    free(G);
    if (rc != 0)
        return rc;
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t j = 0; j < n; ++j) {
            double v = A[r * n + j];
            for (int64_t k = 0; k < j; ++k)
                v -= Q[r * n + k] * R[k * n + j];
            Q[r * n + j] = v / R[j * n + j];
        }
    }
    return 0;
}

int oracle_cholqr(int64_t m, int64_t n, const double *A, double *Q, double *R, int passes)
{
    if (m < 0 || n < 0 || m < n || passes < 1 || passes > 2)
        return -1;
    int rc = cholqr_pass(m, n, A, Q, R);
    if (rc != 0 || passes == 1)
        return rc;
    double *Q1 = (double *)malloc((size_t)(m * n > 0 ? m * n : 1) * sizeof(double));
    double *R1 = (double *)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(double));
    if (!Q1 || !R1) {
        free(Q1);
        free(R1);
        return -2;
    }
    memcpy(Q1, Q, (size_t)(m * n) * sizeof(double));
    memcpy(R1, R, (size_t)(n * n) * sizeof(double));
    double *R2 = (double *)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(double));
    if (!R2) {
        free(Q1);
        free(R1);
        return -2;
    }
    rc = cholqr_pass(m, n, Q1, Q, R2);
    if (rc == 0) {
        /* R = R2 R1, both upper triangular */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double v = 0.0;
                for (int64_t l = i; l <= j; ++l)
                    v += R2[i * n + l] * R1[l * n + j];
                R[i * n + j] = (j >= i) ? v : 0.0;
            }
    }
    free(Q1);
    free(R1);
    free(R2);
    return rc;
}

/*
 * Blocked Householder QR: the same factorisation as oracle_geqrf, organised
 * as in LAPACK xGEQRF (right-looking, panels of nb columns).  This is the
 * conventional QR that CAQR reorganises (Sec. 3: CAQR is blocked Householder
 * QR whose panels are factored by TSQR, with the trailing matrix updated by
 * the panel's reflectors), used as the reference for square matrices too
 * large for the unblocked loop.  Per panel of jb columns starting at column k:
 *  1. Householder QR of the panel A[k:m, k:k+jb] (geqr2_cm, pairwise sums);
 *  2. T, the jb x jb upper triangular factor of the compact form
 *     H_k ... H_{k+jb-1} = I - V T V^T (Schreiber and Van Loan, cited in
 *     Sec. 2.1), by the forward recurrence T[j][j] = tau_j,
 *     T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j), the inner products by
 *     pairwise sums;
 *  3. the trailing columns C = A[k:m, k+jb:n] <- Q_panel^T C
 *     = C - V (T^T (V^T C)): W = V^T C, U = T^T W, C -= V U, each entry a
 *     plain sum in index order.  The columns of C are shared among OpenMP
 *     threads in blocks; every entry is computed by one thread in a fixed
 *     order, so the result does not depend on the thread count.
 * In exact arithmetic the result equals oracle_geqrf's (same reflectors, same
 * tau, same R); in floating point only the summation order of step 3
 * differs.  A: m x n row-major (m >= n), overwritten as by oracle_geqrf;
 * tau: n entries; nb >= 1.  Returns 0, -1 for bad sizes, -2 on allocation
 * failure.
 */
int oracle_geqrf_blocked(int64_t m, int64_t n, double *A, double *tau, int64_t nb)
{
    if (m < 0 || n < 0 || m < n || nb < 1)
        return -1;
    if (n == 0)
        return 0;
    const int64_t bmax = nb < n ? nb : n;
    double *P = (double *)malloc((size_t)(m * bmax) * sizeof(double));   /* panel, column-major */
    double *Vr = (double *)malloc((size_t)(m * bmax) * sizeof(double));  /* V, row-major */
    double *T = (double *)malloc((size_t)(bmax * bmax) * sizeof(double));
    scratch_t s = {0, 0};
    if (!P || !Vr || !T || scratch_reserve(&s, m) != 0) {
        free(P);
        free(Vr);
        free(T);
        free(s.p);
        return -2;
    }
    int rc = 0;
    for (int64_t k = 0; k < n && rc == 0; k += nb) {
        const int64_t jb = (n - k) < nb ? (n - k) : nb;
        const int64_t mk = m - k;
        /* 1. the panel */
        for (int64_t i = 0; i < mk; ++i)
            for (int64_t j = 0; j < jb; ++j)
                P[j * mk + i] = A[(k + i) * n + k + j];
        if (geqr2_cm(mk, jb, P, tau + k) != 0) {
            rc = -2;
            break;
        }
        for (int64_t i = 0; i < mk; ++i)
            for (int64_t j = 0; j < jb; ++j)
                A[(k + i) * n + k + j] = P[j * mk + i];
        if (k + jb >= n)
            break;
        /* V row-major: unit diagonal, zeros above it */
        for (int64_t i = 0; i < mk; ++i)
            for (int64_t j = 0; j < jb; ++j)
                Vr[i * jb + j] = (i > j) ? P[j * mk + i] : ((i == j) ? 1.0 : 0.0);
        /* 2. T by the forward recurrence */
        for (int64_t j = 0; j < jb; ++j) {
            for (int64_t i = 0; i < jb; ++i)
                T[i * jb + j] = 0.0;
            T[j * jb + j] = tau[k + j];
            if (tau[k + j] == 0.0)
                continue;
            for (int64_t l = 0; l < j; ++l) {
                /* (V[:, l]^T v_j): rows i >= j, V[j][l] * 1 plus the tails */
                const int64_t len = mk - j;
                s.p[0] = P[l * mk + j];
                for (int64_t i = 1; i < len; ++i)
                    s.p[i] = P[l * mk + j + i] * P[j * mk + j + i];
                T[l * jb + j] = psum(s.p, len); /* z_l, scaled below */
            }
            /* T[0:j, j] = -tau_j T[0:j, 0:j] z, rows in order (T upper) */
            for (int64_t l = 0; l < j; ++l) {
                double acc = 0.0;
                for (int64_t q = l; q < j; ++q)
                    acc += T[l * jb + q] * T[q * jb + j];
                s.p[l] = -tau[k + j] * acc;
            }
            for (int64_t l = 0; l < j; ++l)
                T[l * jb + j] = s.p[l];
        }
        /* 3. trailing columns, in blocks of CB per thread */
        const int64_t c0 = k + jb, nc = n - c0;
        enum { CB = 32 };
        const int64_t nblk = (nc + CB - 1) / CB;
        int fail = 0;
#pragma omp parallel
        {
            double *W = (double *)malloc((size_t)(jb * CB) * sizeof(double));
            double *U = (double *)malloc((size_t)(jb * CB) * sizeof(double));
            if (!W || !U) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(dynamic, 1)
            for (int64_t bk = 0; bk < nblk; ++bk) {
                if (!W || !U)
                    continue;
                const int64_t cs = c0 + bk * CB;
                const int64_t w = (n - cs) < CB ? (n - cs) : CB;
                double srow[CB];
                /* W = V^T C */
                for (int64_t e = 0; e < jb * CB; ++e)
                    W[e] = 0.0;
                for (int64_t i = 0; i < mk; ++i) {
                    const double *a = A + (k + i) * n + cs;
                    const double *v = Vr + i * jb;
                    for (int64_t j = 0; j < jb; ++j) {
                        const double vij = v[j];
                        double *wr = W + j * CB;
                        for (int64_t c = 0; c < w; ++c)
                            wr[c] += vij * a[c];
                    }
                }
                /* U = T^T W: U[j][c] = sum_{l <= j} T[l][j] W[l][c] */
                for (int64_t j = 0; j < jb; ++j) {
                    double *ur = U + j * CB;
                    for (int64_t c = 0; c < w; ++c)
                        ur[c] = 0.0;
                    for (int64_t l = 0; l <= j; ++l) {
                        const double t = T[l * jb + j];
                        const double *wr = W + l * CB;
                        for (int64_t c = 0; c < w; ++c)
                            ur[c] += t * wr[c];
                    }
                }
                /* C -= V U, row by row */
                for (int64_t i = 0; i < mk; ++i) {
                    double *a = A + (k + i) * n + cs;
                    const double *v = Vr + i * jb;
                    for (int64_t c = 0; c < w; ++c)
                        srow[c] = 0.0;
                    for (int64_t j = 0; j < jb; ++j) {
                        const double vij = v[j];
                        const double *ur = U + j * CB;
                        for (int64_t c = 0; c < w; ++c)
                            srow[c] += vij * ur[c];
                    }
                    for (int64_t c = 0; c < w; ++c)
                        a[c] -= srow[c];
                }
            }
            free(W);
            free(U);
        }
        if (fail)
            rc = -2;
    }
    free(P);
    free(Vr);
    free(T);
    free(s.p);
    return rc;
}

/*
 * Modified Gram-Schmidt, the other unstable alternative of the paper's
 * comparison (Sec. 2.3, with CholeskyQR; its loss of orthogonality grows with
 * the condition number).  Textbook right-looking form: for j = 0..n-1,
 * R_jj = ||a_j||, q_j = a_j / R_jj, then for every later column c,
 * R_jc = q_j^T a_c and a_c -= R_jc q_j (a_c being the column as already
 * updated by q_0..q_{j-1}).  Sums over the m rows are pairwise.
 * Inputs row-major: A m x n.  Outputs: Q m x n, R n x n (zeros below the
 * diagonal).  Returns 0, -1 for bad sizes, -2 on allocation failure, -3 if a
 * column becomes exactly zero (rank deficiency: R_jj = 0).
 */
int oracle_mgs(int64_t m, int64_t n, const double *A, double *Q, double *R)
{
    if (m < 0 || n < 0 || m < n)
        return -1;
    double *ac = to_cm(m, n, A);
    scratch_t s = {0, 0};
    if (!ac || scratch_reserve(&s, m > 0 ? m : 1) != 0) {
        free(ac);
        free(s.p);
        return -2;
    }
    memset(R, 0, (size_t)(n * n) * sizeof(double));
    int rc = 0;
    for (int64_t j = 0; j < n; ++j) {
        double *q = ac + j * m;
        double nrm = sqrt(pdot(&s, q, q, m));
        if (nrm == 0.0) {
            rc = -3;
            break;
        }
        R[j * n + j] = nrm;
        for (int64_t i = 0; i < m; ++i)
            q[i] /= nrm;
        for (int64_t c = j + 1; c < n; ++c) {
            double *a = ac + c * m;
            double r = pdot(&s, q, a, m);
            R[j * n + c] = r;
            for (int64_t i = 0; i < m; ++i)
                a[i] -= r * q[i];
        }
    }
    if (rc == 0)
        from_cm(m, n, ac, Q);
    free(ac);
    free(s.p);
    return rc;
}

/* Number of OpenMP threads for later calls (<= 0: the runtime's default);
 * returns the number the runtime will use. */
int oracle_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Exposed for the tests: pairwise sum of n doubles. */
double oracle_psum(const double *x, int64_t n) { return psum(x, n); }
