"""Graded reference: the exact ridge path by one Cholesky solve per lambda.

For every lam in the grid and every right-hand side column,
    x*(lam) = (A^T A + lam I)^-1 A^T b           (Section 1, Eq. (least-square);
                                                    the same quantity as the
                                                    closed form of Section 2.1)
computed in FP64 from the exact FP64 values of the input bytes: G = A^T A
and C = A^T B are formed once, then for each lam the Cholesky factor of
G + lam I solves for the d x K block.  Matrix right-hand sides follow the
matrix-valued problem Eq. (least-square-max) of Section 5.3, column by column.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _is_csr(A):
    return hasattr(A, "row_ptr")


def _sparse64(A):
    return sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr),
                         shape=(A.n, A.d))


def gram(A, chunk: int = 1 << 14) -> np.ndarray:
    """G = A^T A in FP64 (row chunks are upcast one at a time)."""
    if _is_csr(A):
        S = _sparse64(A)
        return np.asarray((S.T @ S).todense())
    n, d = A.shape
    G = np.zeros((d, d))
    for r0 in range(0, n, chunk):
        blk = np.asarray(A[r0:r0 + chunk], dtype=np.float64)
        G += blk.T @ blk
    return G


def atb(A, B, chunk: int = 1 << 14) -> np.ndarray:
    """C = A^T B in FP64 (d x K)."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    if _is_csr(A):
        return np.asarray(_sparse64(A).T @ B)
    n, d = A.shape
    C = np.zeros((d, B.shape[1]))
    for r0 in range(0, n, chunk):
        C += np.asarray(A[r0:r0 + chunk], dtype=np.float64).T @ B[r0:r0 + chunk]
    return C


def solve_from_gram(G: np.ndarray, C: np.ndarray, lambdas) -> np.ndarray:
    """X[t] = (G + lambdas[t] I)^-1 C for every t; returns T x d x K."""
    lambdas = np.atleast_1d(np.asarray(lambdas, dtype=np.float64))
    d = G.shape[0]
    out = np.empty((len(lambdas), d, C.shape[1]))
    for t, lam in enumerate(lambdas):
        H = G.copy()
        H[np.diag_indices(d)] += lam
        out[t] = sla.cho_solve(sla.cho_factor(H, lower=True, check_finite=False), C,
                               check_finite=False)
    return out


def ridge_path(A, B, lambdas) -> np.ndarray:
    """The exact ridge path, T x d x K, FP64."""
    return solve_from_gram(gram(A), atb(A, B), lambdas)


def dual_gram(A, chunk: int = 1 << 14) -> np.ndarray:
    """A A^T in FP64 (n x n), formed column chunk by column chunk."""
    A64 = np.asarray(A, dtype=np.float64)
    n, d = A64.shape
    K = np.zeros((n, n))
    for c0 in range(0, d, chunk):
        blk = A64[:, c0:c0 + chunk]
        K += blk @ blk.T
    return K


def solve_dual_from_gram(Kmat: np.ndarray, A, B, lambdas) -> np.ndarray:
    """X[t] = A^T (Kmat + lambdas[t] I)^-1 B with Kmat = A A^T; T x d x K."""
    A64 = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, d = A64.shape
    lambdas = np.atleast_1d(np.asarray(lambdas, dtype=np.float64))
    out = np.empty((len(lambdas), d, B.shape[1]))
    for t, lam in enumerate(lambdas):
        H = Kmat.copy()
        H[np.diag_indices(n)] += lam
        Z = sla.cho_solve(sla.cho_factor(H, lower=True, check_finite=False), B,
                          check_finite=False)
        out[t] = A64.T @ Z
    return out


def ridge_path_dual(A, B, lambdas) -> np.ndarray:
    """The same exact path for n < d through the dual problem of Section 5.2:
    x*(lam) = A^T (A A^T + lam I)^-1 b (the dual optimality condition and the
    primal map x = A^T z).  Returns T x d x K."""
    return solve_dual_from_gram(dual_gram(A), A, B, lambdas)


def solve_from_eig(evals: np.ndarray, V: np.ndarray, C: np.ndarray, lambdas) -> np.ndarray:
    """X[t] = V diag(1 / (evals + lambdas[t])) V^T C; returns T x d x K.

    With G = A^T A = V diag(sigma^2) V^T and C = A^T B = V diag(sigma) U^T B
    this is the closed form x*(lam) = V diag(sigma / (sigma^2 + lam)) U^T b of
    Section 2.1 (one eigendecomposition of G serves every lambda, O(d^2 K)
    per lambda afterwards).  ``eig_of_gram`` gives evals, V."""
    lambdas = np.atleast_1d(np.asarray(lambdas, dtype=np.float64))
    W = V.T @ np.asarray(C, dtype=np.float64)
    out = np.empty((len(lambdas), V.shape[0], W.shape[1]))
    for t, lam in enumerate(lambdas):
        out[t] = V @ (W / (evals + lam)[:, None])
    return out


def eig_of_gram(G: np.ndarray):
    """Eigenvalues (clipped at 0: G is PSD) and eigenvectors of G = A^T A."""
    evals, V = np.linalg.eigh(G)
    return np.maximum(evals, 0.0), V


def ridge_path_eig(A, B, lambdas) -> np.ndarray:
    """The exact ridge path through the eigendecomposition of G (Section 2.1),
    T x d x K, FP64; for many lambdas at large d."""
    evals, V = eig_of_gram(gram(A))
    return solve_from_eig(evals, V, atb(A, B), lambdas)


def rel_err(X_hat, X_ref) -> np.ndarray:
    """Per-lambda relative Frobenius error ||X_hat[t] - X_ref[t]|| / ||X_ref[t]||
    (each of the T leading blocks is one lambda; a block of zeros in X_ref
    gives inf or nan, never a small number)."""
    X_ref = np.asarray(X_ref, dtype=np.float64)
    X_hat = np.asarray(X_hat, dtype=np.float64).reshape(X_ref.shape)
    T = X_ref.shape[0]
    num = np.sqrt(np.sum((X_hat - X_ref).reshape(T, -1) ** 2, axis=1))
    den = np.sqrt(np.sum(X_ref.reshape(T, -1) ** 2, axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        return num / den
