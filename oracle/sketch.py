"""The sketch families of Section 4, built or applied plainly in FP64.

Gaussian    S_ij ~ N(0, 1/m)                         (Section 4, bullet 1);
            its BF16 form rounds the N(0,1) draws to BF16 before the 1/sqrt(m),
            its FP8 form to e4m3 and multiplies A's three-term e4m3 form
CountSketch one +-1 per column of S at a hashed row    (Section 4, bullet 2)
SJLT        s stacked CountSketches of m/s rows each, scaled 1/sqrt(s)
                                                       (Section 4, bullet 3)
SRHT        S = sqrt(n'/m) R (H_n'/sqrt(n')) D with D random signs, H the
            Walsh-Hadamard matrix of order n' = 2^ceil(log2 n) (A padded with
            zero rows) and R m rows sampled uniformly with replacement
                                                       (Section 4, bullet 4)
All draws come from ``oracle.rng``.  The bucket index of CountSketch is taken
in {0..m-1} (the printed range {1..n} cannot index m rows).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import rng


def _dense64(A):
    if hasattr(A, "row_ptr"):
        return sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr),
                             shape=(A.n, A.d)).toarray()
    return np.asarray(A, dtype=np.float64)


def _sparse64(A):
    if hasattr(A, "row_ptr"):
        return sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr),
                             shape=(A.n, A.d))
    return sp.csr_matrix(np.asarray(A, dtype=np.float64))


def countsketch_matrix(seed: int, n: int, m: int, s: int = 1):
    """Sparse S (m x n) of an SJLT with s blocks (s = 1: CountSketch)."""
    h, sg = rng.countsketch_draws(seed, n, m, s)
    cols = np.repeat(np.arange(n), s)
    vals = sg.reshape(-1).astype(np.float64) / np.sqrt(s)
    return sp.csr_matrix((vals, (h.reshape(-1), cols)), shape=(m, n))


def countsketch_apply(A, seed: int, m: int, s: int = 1) -> np.ndarray:
    """S A for CountSketch / SJLT; dense or CSR A, FP64 result (m x d)."""
    S = countsketch_matrix(seed, A.shape[0], m, s)
    return np.asarray((S @ _sparse64(A)).todense())


def fwht(X: np.ndarray) -> np.ndarray:
    """Unnormalized Walsh-Hadamard transform along axis 0 (length 2^p).

    Sylvester order: (H x)_r = sum_i (-1)^popcount(r & i) x_i, computed by
    p rounds of sum/difference butterflies.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    h = 1
    while h < n:
        Y = X.reshape(n // (2 * h), 2, h, *X.shape[1:])
        a = Y[:, 0].copy()
        b = Y[:, 1].copy()
        Y[:, 0] = a + b
        Y[:, 1] = a - b
        X = Y.reshape(X.shape)
        h *= 2
    return X


def srht_apply(A, seed: int, m: int) -> np.ndarray:
    """S A for the SRHT, FP64 result (m x d)."""
    A64 = _dense64(A)
    n, d = A64.shape
    signs, rows, npad = rng.srht_draws(seed, n, m)
    Z = np.zeros((npad, d))
    Z[:n] = signs.astype(np.float64)[:, None] * A64
    Z = fwht(Z)
    return Z[rows] / np.sqrt(m)


def srht_matrix(seed: int, n: int, m: int) -> np.ndarray:
    """Dense S (m x n) of the SRHT, for tiny n only."""
    from scipy.linalg import hadamard
    signs, rows, npad = rng.srht_draws(seed, n, m)
    H = hadamard(npad).astype(np.float64)
    return H[rows][:, :n] * signs.astype(np.float64)[None, :] / np.sqrt(m)


def gaussian_apply(A, seed: int, m: int) -> np.ndarray:
    """S A for the Gaussian sketch, FP64 result (m x d)."""
    S = rng.gaussian_matrix(seed, m, A.shape[0])
    if hasattr(A, "row_ptr"):
        return np.asarray((_sparse64(A).T @ S.T).T)
    return S @ np.asarray(A, dtype=np.float64)


def gaussian_bf16_apply(A, seed: int, m: int) -> np.ndarray:
    """S A for the BF16 Gaussian sketch S = BF16(FP32(z)) / sqrt(m), FP64."""
    S = rng.gaussian_matrix_bf16(seed, m, A.shape[0])
    return S @ np.asarray(A, dtype=np.float64)


def fp8_column_exponents(A) -> np.ndarray:
    """Per column c the smallest integer e_c with max_k |a_kc| <= 448 * 2^e_c
    (0 for a column of zeros): the power-of-two scale that brings the
    column's largest entry to the top binade of e4m3."""
    mx = np.abs(np.asarray(A, dtype=np.float64)).max(axis=0)
    e = np.zeros(mx.shape, dtype=np.int64)
    for c, v in enumerate(mx):
        if v > 0:
            k = int(np.floor(np.log2(v))) - 8
            while v > np.ldexp(448.0, k):
                k += 1
            while v <= np.ldexp(448.0, k - 1):
                k -= 1
            e[c] = k
    return e


def fp8_terms(A):
    """A split into three e4m3 terms under the per-column scale 2^e_c: with
    r_0 = A 2^-e, t_p = E4M3(r_p) and r_{p+1} = 16 (r_p - t_p),
    A ~ 2^e (t_0 + t_1/16 + t_2/256).  Returns (t (3 x n x d), e)."""
    e = fp8_column_exponents(A)
    r = np.ldexp(np.asarray(A, dtype=np.float64), -e[None, :])
    t = []
    for _ in range(3):
        tp = rng.round_e4m3(r)
        t.append(tp)
        r = (r - tp) * 16.0
    return np.stack(t), e


def fp8_reconstruct(A) -> np.ndarray:
    """The FP8 form of A the FP8 sketch multiplies: 2^e (t_0 + t_1/16 + t_2/256)."""
    t, e = fp8_terms(A)
    return np.ldexp(t[0] + t[1] / 16.0 + t[2] / 256.0, e[None, :])


def gaussian_fp8_apply(A, seed: int, m: int) -> np.ndarray:
    """S A for the FP8 Gaussian sketch: S = E4M3(FP32(z)) / sqrt(m) applied to
    the three-term e4m3 form of A, FP64."""
    S = rng.gaussian_matrix_fp8(seed, m, A.shape[0])
    return S @ fp8_reconstruct(A)


def apply(kind: str, A, seed: int, m: int, s: int = 1) -> np.ndarray:
    if kind == "gaussian":
        return gaussian_apply(A, seed, m)
    if kind == "srht":
        return srht_apply(A, seed, m)
    if kind == "countsketch":
        return countsketch_apply(A, seed, m, 1)
    if kind == "sjlt":
        return countsketch_apply(A, seed, m, s)
    raise ValueError(kind)
