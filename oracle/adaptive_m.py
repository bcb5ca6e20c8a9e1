"""Adaptive sketch dimension (Section 5.1, Algorithm 4) in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

IHS at lam = lam_min with a backtracking line search, doubling m whenever
the progress measure stalls:

    f(X)     = 1/2 ||A X - B||_F^2 + lam/2 ||X||_F^2
    grad f   = A^T (A X - B) + lam X
    D_k      = (A^T S^T S A + lam I)^-1 grad f(X_k)
    delta_k  = <D_k, grad f(X_k)>                    (trace form for K > 1)
    tau_k    = gamma1^j, j >= 0 the smallest with
               f(X_k - tau D_k) <= f(X_k) - gamma2 tau delta_k   (Eq. (armijo))
    X_{k+1}  = X_k - tau_k D_k

Readings taken where the text is garbled or silent:
* the gradient is A^T (A x - b) + lam x (the printed A^T (A x - b + lam x)
  does not type-check for n != d);
* the test that doubles m sits inside the loop, after each update: with
  delta_{k+1} computed from the current sketch, delta_{k+1} >= gamma3 delta_k
  doubles m, redraws S at the new size and recomputes D_{k+1}, delta_{k+1}
  at the new iterate X_{k+1} (the step taken is kept: Armijo made it a
  descent step);
* the stop test compares with the first value: delta_k <= eps * delta_0
  (the printed eps is absolute; the relative form is scale free);
* X_0 = 0; m never exceeds m_cap, and once it is there no more doublings
  happen; a sketch of m >= n rows is replaced by S = I (the exact Hessian);
  an SJLT's m is kept a multiple of its s;
* S is redrawn from the same seed at the new size (``oracle.sketch``
  draws depend on (seed, m)).
The defaults gamma1 = 0.5, gamma2 = 1e-4, gamma3 = 0.5 are this module's
choice (the text leaves them open).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import direct, sketch


@dataclass
class Alg4Result:
    m: int                      # the sketch dimension the algorithm ends with
    X: np.ndarray               # the last iterate (d x K)
    iters: int                  # IHS updates taken
    doublings: int
    # one row per update k: (m in effect, tau_k, delta_k, delta_{k+1} from the
    # same sketch, 1 if m doubled after it)
    trace: list = field(default_factory=list)
    iterates: list = field(default_factory=list)   # X_0 .. X_iters (keep_iterates)


def _dense_or_sparse(A):
    if hasattr(A, "row_ptr"):
        return direct._sparse64(A)
    return np.asarray(A, dtype=np.float64)


def sketch_size(A, B, lam: float, kind: str, seed: int, m0: int, *, dual: bool = False,
                s: int = 1, m_cap: int | None = None, gamma1: float = 0.5,
                gamma2: float = 1e-4, gamma3: float = 0.5, eps: float = 1e-8,
                max_iter: int = 50, max_armijo: int = 60,
                keep_iterates: bool = False) -> Alg4Result:
    """Algorithm 4 for f at lam (= lam_min); returns the final m and a trace.

    dual=True (n < d, dense A): the same search on the dual problem of
    Section 5.2, Eq. (ls_reg:d), f(z) = 1/2 ||A^T z||^2 + lam/2 ||z||^2 - <B, z>,
    whose Hessian A A^T + lam I is sketched as (S A^T)^T (S A^T) + lam I; X is
    then the dual iterate z (n x K).
    """
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    if dual:
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)  # the d x n matrix A^T
    Ad = _dense_or_sparse(A)
    n, d = Ad.shape
    if m_cap is None:
        m_cap = n

    if dual:
        def f(X):
            R = Ad @ X
            return (0.5 * float(np.sum(R * R)) + 0.5 * lam * float(np.sum(X * X))
                    - float(np.sum(B * X)))

        def grad(X):
            return np.asarray(Ad.T @ (Ad @ X)) + lam * X - B
    else:
        def f(X):
            R = Ad @ X - B
            return 0.5 * float(np.sum(R * R)) + 0.5 * lam * float(np.sum(X * X))

        def grad(X):
            return np.asarray(Ad.T @ (Ad @ X - B)) + lam * X

    def precond(m):
        if m >= n:
            SA = Ad.toarray() if hasattr(Ad, "toarray") else Ad
        else:
            SA = sketch.apply(kind, A, seed, m, s)
        H = np.asarray(SA.T @ SA)
        H[np.diag_indices(d)] += lam
        cf = sla.cho_factor(H, lower=True)
        return lambda V: sla.cho_solve(cf, V)

    m = int(m0)
    P = precond(m)
    X = np.zeros((d, B.shape[1]))
    g = grad(X)
    D = P(g)
    delta = float(np.sum(D * g))
    delta0 = delta
    res = Alg4Result(m=m, X=X, iters=0, doublings=0)
    if keep_iterates:
        res.iterates.append(X.copy())
    k = 0
    while delta > eps * delta0 and k < max_iter:
        fx = f(X)
        tau = 1.0
        for _ in range(max_armijo):
            if f(X - tau * D) <= fx - gamma2 * tau * delta:
                break
            tau *= gamma1
        else:
            raise RuntimeError("Armijo search failed")
        X = X - tau * D
        if keep_iterates:
            res.iterates.append(X.copy())
        g = grad(X)
        D = P(g)
        delta_next = float(np.sum(D * g))
        m_step, doubled = m, 0
        if delta_next >= gamma3 * delta and m < m_cap:
            m_new = min(2 * m, m_cap)
            if s > 1 and m_new < n:
                m_new -= m_new % s      # SJLT needs s | m
            if m_new > m:
                m = m_new
                P = precond(m)
                D = P(g)
                doubled = 1
                res.doublings += 1
        res.trace.append((m_step, tau, delta, delta_next, doubled))
        delta = float(np.sum(D * g))
        k += 1
    res.m, res.X, res.iters = m, X, k
    return res
