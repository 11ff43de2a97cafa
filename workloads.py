"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and shapes them; it holds none of the
factorisation's arithmetic.  The workloads follow the shapes and value
distributions of the measured configurations (iid N(0,1) entries; one
ill-conditioned matrix with log-spaced singular values).  The paper uses no
public dataset, so everything here is synthetic.

All draws use ``numpy.random.default_rng(seed)`` (PCG64) in FP64; FP32
inputs are the FP64 draws rounded to FP32.
"""
from __future__ import annotations

import numpy as np


def gaussian(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """m x n matrix with iid N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)).astype(dtype)


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    """Random n x n orthogonal matrix: the orthogonal factor of an n x n
    Gaussian (LAPACK QR via numpy), with columns scaled by sign(diag R) so
    that the distribution is the Haar measure."""
    G = gaussian(n, n, seed)
    Qw, Rw = np.linalg.qr(G)
    d = np.sign(np.diag(Rw))
    d[d == 0] = 1.0
    return Qw * d[None, :]


def logspace_sv(n: int, cond: float) -> np.ndarray:
    """s_i = cond^(-i/(n-1)), i = 0..n-1 (from 1 down to 1/cond)."""
    if n == 1:
        return np.ones(1)
    return cond ** (-np.arange(n) / (n - 1.0))


def conditioned(m: int, n: int, cond: float, seed_g: int, seed_w: int) -> np.ndarray:
    """A = G diag(s) W with G Gaussian (seed_g), s log-spaced from 1 to
    1/cond and W Haar orthogonal (seed_w)."""
    G = gaussian(m, n, seed_g)
    s = logspace_sv(n, cond)
    W = haar_orthogonal(n, seed_w)
    return (G * s[None, :]) @ W


# ---- the measured configurations, with their seeds ----

def cfg1():
    """Plain TSQR, FP64: one 4096 x 16 Gaussian matrix (seed 1)."""
    return gaussian(4096, 16, 1)


def cfg2(m: int = 1 << 20, n: int = 64, k: int = 32):
    """Bandwidth-bound TSQR, FP64: A = G diag(s) W, G m x n Gaussian (seed 2),
    s log-spaced 1..1e-8, W Haar (seed 3); B m x k Gaussian (seed 4)."""
    A = conditioned(m, n, 1e8, 2, 3)
    B = gaussian(m, k, 4)
    return A, B


def cfg3(n: int = 16384):
    """CAQR: n x n Gaussian (seed 5)."""
    return gaussian(n, n, 5)


def cfg4_shapes(count: int = 2000, seed: int = 6, m_lo: int = 512, m_hi: int = 65536,
                n_choices=(8, 16, 32, 64)):
    """Batched uneven TSQR: m ~ U{m_lo..m_hi}, n ~ U(n_choices)."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def cfg4_matrix(i: int, m: int, n: int, seed: int = 6, dtype=np.float64) -> np.ndarray:
    """Entries of matrix i of the batch: iid N(0,1), seeded by (seed, i)."""
    rng = np.random.default_rng([seed, i])
    return rng.standard_normal((m, n)).astype(dtype)


def cfg5(m: int = 262144, n: int = 32):
    """Differentiable TSQR, FP64: A (seed 7), upstream dQ (seed 8), dR (seed 9)."""
    return gaussian(m, n, 7), gaussian(m, n, 8), gaussian(n, n, 9)


def cfg5_batch(batch: int = 256, m: int = 8192, n: int = 32):
    """FP32 batch for the differentiable TSQR (seed 10): A, dQ, dR."""
    rng = np.random.default_rng(10)
    A = rng.standard_normal((batch, m, n)).astype(np.float32)
    dQ = rng.standard_normal((batch, m, n)).astype(np.float32)
    dR = rng.standard_normal((batch, n, n)).astype(np.float32)
    return A, dQ, dR


def fd_case(m: int = 1024, n: int = 8):
    """Finite-difference check case (seed 11)."""
    return gaussian(m, n, 11)


def cfg4_device_matrix(i: int, m: int, n: int, seed: int = 6, dtype=None, device="cuda"):
    """Matrix i of the batch generated on the device (iid N(0,1), torch's
    Philox generator seeded by seed * 1000003 + i): the full 2000-matrix batch
    (about 16 GB in FP64) is drawn on the GPU; tests copy the matrices they
    check back to the host."""
    import torch
    g = torch.Generator(device=device).manual_seed(seed * 1000003 + i)
    return torch.randn(m, n, dtype=dtype or torch.float64, device=device, generator=g)
