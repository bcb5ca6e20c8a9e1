"""IHS-BIN in FP64, step by step in the paper's order (diagnostic oracle).

Notation follows Section 4.  For an interval [lo, hi] with centre lam0:
    P_S = (A^T S^T S A + lam0 I)^-1                                 (Section 4)
    M(lam) = I - tau P_S (A^T A + lam I)                    (Eq. (equ:ihs))
    x_k(lam) = tau sum_{i<k} M(lam)^i P_S A^T b
             = tau sum_{j<k} (tau (lam - ref))^j  ut_j              (Proposition)
with ut_j = sum_{i>=j} u_{i,j} and the recursion Eq. (equ:upd)
    u_{0,0} = P_S A^T b,
    u_{i+1,0} = (I - tau P_S H) u_{i,0},
    u_{i+1,j} = (I - tau P_S H) u_{i,j} - P_S u_{i,j-1},   1 <= j <= i,
    u_{i+1,i+1} = -P_S u_{i,i},
where H = A^T A + ref I.  ``ref = 0`` is the printed expansion (powers of
tau*lam); ``ref = lam0`` expands the same polynomial about the interval
centre, M(lam) = (I - tau P_S (A^T A + lam0 I)) - tau (lam - lam0) P_S, whose
terms do not grow with i.  Both give the same x_k(lam) in exact arithmetic.

Readings taken where the text is ambiguous:
* the seed is u_{0,0} = +P_S A^T b as in the Proposition (Algorithm 2 prints
  a minus sign, which together with Algorithm 3 would return -x);
* the basis is built once per interval, outside the loop over lambda
  (Algorithm 3 places it inside the loop but prices it once);
* L = floor(2 ln(lam_max / lam_min)) intervals (natural log), boundaries
  lam^(l) = lam_min * beta^(l/L), centre lam0 = sqrt(lam^(l) lam^(l+1))
  (Section 4.2 and Theorem 1); a lambda on a boundary belongs to the lower
  interval;
* step size: the proof of Theorem 1 bounds the spectrum of P_S (A^T A + lam I)
  over the whole interval and picks tau = 2 / (c_min + c_max), the minimizer
  of max |1 - tau c| over [c_min, c_max]; the rate is
  r = (c_max - c_min)/(c_max + c_min).  The bounds used here are the exact
  ones over the interval: in the symmetric form L^-1 (A^T A + lam I) L^-T =
  B_0 + lam L^-1 L^-T (P_S = L^-T L^-1) each Rayleigh quotient grows with
  lam, so the smallest eigenvalue over [lo, hi] is the one at lo and the
  largest the one at hi: c_min = lambda_min(P_S (A^T A + lo I)),
  c_max = lambda_max(P_S (A^T A + hi I)).  (``step_size`` keeps the looser
  form [mu_min lo/lam0, mu_max hi/lam0] built from the spectrum at lam0,
  which with the theoretical bounds mu = 1/rho reproduces Theorem 1's alpha.)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import direct


# ---------------------------------------------------------------- plan (4.2)
def num_intervals(lam_min: float, lam_max: float) -> int:
    """L = floor(2 ln beta), at least 1 (Section 4.2, Section 6.1)."""
    beta = lam_max / lam_min
    return max(1, int(math.floor(2.0 * math.log(beta)))) if beta > 1 else 1


def plan(lam_min: float, lam_max: float, L: int | None = None, sigma_d2: float = 0.0):
    """Interval boundaries lam^(0..L) and centres lam0^(0..L-1).

    With sigma_d2 = sigma_d^2 > 0 (the smallest squared singular value of A,
    or an estimate) the centre of [lo, hi] follows the remark after Theorem 1:
    lam0 = sqrt((hi + s)(lo + s)) - s, the shift whose (lam0 + s) is the
    geometric centre of (lo + s, hi + s); s = 0 gives sqrt(lo hi).  It is
    evaluated as (lo hi + s (lo + hi)) / (sqrt((lo + s)(hi + s)) + s), the same
    number without the cancellation of the difference when s >> hi.
    """
    if not (lam_min > 0 and lam_max >= lam_min):
        raise ValueError("need 0 < lam_min <= lam_max")
    if not sigma_d2 >= 0:
        raise ValueError("need sigma_d2 >= 0")
    L = L or num_intervals(lam_min, lam_max)
    beta = lam_max / lam_min
    grid = np.array([lam_min * beta ** (l / L) for l in range(L + 1)])
    grid[-1] = lam_max
    s = float(sigma_d2)
    lo, hi = grid[:-1], grid[1:]
    lam0 = (lo * hi + s * (lo + hi)) / (np.sqrt((lo + s) * (hi + s)) + s)
    return grid, lam0


def interval_of(lam: float, grid: np.ndarray) -> int:
    """Index l with grid[l] <= lam <= grid[l+1]; boundaries go to the lower one."""
    L = len(grid) - 1
    l = int(np.searchsorted(grid[1:], lam, side="left"))
    return min(max(l, 0), L - 1)


# ------------------------------------------------------- operators (Section 4)
class Operator:
    """A^T A v for dense or CSR A, in FP64, without forming A^T A."""

    def __init__(self, A):
        if hasattr(A, "row_ptr"):
            self._A = direct._sparse64(A)
        else:
            self._A = np.asarray(A, dtype=np.float64)

    def AtA(self, V):
        return self._A.T @ (self._A @ V)

    def At(self, B):
        return self._A.T @ np.asarray(B, dtype=np.float64)

    def dense_gram(self):
        G = self._A.T @ self._A
        return np.asarray(G.todense()) if hasattr(G, "todense") else G


class Precond:
    """P_S = (SA^T SA + lam0 I)^-1 applied through its Cholesky factor."""

    def __init__(self, SA: np.ndarray, lam0: float):
        GS = SA.T @ SA
        GS[np.diag_indices_from(GS)] += lam0
        self.lam0 = lam0
        self.chol = sla.cho_factor(GS, lower=True)

    def __call__(self, V):
        return sla.cho_solve(self.chol, V)

    def factor(self) -> np.ndarray:
        return np.tril(self.chol[0])


def spectrum_bounds(op: Operator, P: Precond):
    """Exact extreme eigenvalues of P_S (A^T A + lam0 I) (dense, small d only)."""
    Lf = P.factor()
    H = op.dense_gram()
    H[np.diag_indices_from(H)] += P.lam0
    X = sla.solve_triangular(Lf, H, lower=True)
    Bm = sla.solve_triangular(Lf, X.T, lower=True)
    ev = np.linalg.eigvalsh(0.5 * (Bm + Bm.T))
    return float(ev[0]), float(ev[-1])


def spectrum_at(op: Operator, P: Precond, lam: float):
    """Exact extreme eigenvalues of P_S (A^T A + lam I) (dense, small d only)."""
    Lf = P.factor()
    H = op.dense_gram()
    H[np.diag_indices_from(H)] += lam
    X = sla.solve_triangular(Lf, H, lower=True)
    Bm = sla.solve_triangular(Lf, X.T, lower=True)
    ev = np.linalg.eigvalsh(0.5 * (Bm + Bm.T))
    return float(ev[0]), float(ev[-1])


def interval_bounds(op: Operator, P: Precond, lo: float, hi: float):
    """[c_min, c_max] holding the spectrum of P_S (A^T A + lam I) for every
    lam in [lo, hi]: the smallest eigenvalue at lo, the largest at hi."""
    return spectrum_at(op, P, lo)[0], spectrum_at(op, P, hi)[1]


def step_size_from_bounds(cmin: float, cmax: float):
    """tau = 2 / (c_min + c_max) and the rate (c_max - c_min) / (c_max + c_min)."""
    return 2.0 / (cmin + cmax), (cmax - cmin) / (cmax + cmin)


def step_size(mu_min: float, mu_max: float, lo: float, hi: float, lam0: float):
    """tau and predicted rate for the interval [lo, hi] (see module notes)."""
    cmin = mu_min * lo / lam0
    cmax = mu_max * hi / lam0
    return 2.0 / (cmin + cmax), (cmax - cmin) / (cmax + cmin)


# -------------------------------- basis (the Proposition, Eq. (equ:upd))
def recursion_step(u, P, Hop, tau: float):
    """One whole step of Eq. (equ:upd): from u_{i,0..i} to u_{i+1,0..i+1}.

    u_{i+1,j} = u_{i,j} - P_S (tau H u_{i,j} + u_{i,j-1}), where a term whose
    index falls outside 0..i is zero: j = 0 has no u_{i,-1}, and j = i+1 has
    no u_{i,i+1}, which leaves u_{i+1,i+1} = -P_S u_{i,i}.  Every new vector
    reads only step-i vectors.  H = A^T A + ref I (``Hop``)."""
    i = len(u) - 1
    new = []
    for j in range(i + 2):
        prev = u[j] if j <= i else None
        lower = u[j - 1] if j >= 1 else None
        rhs = tau * Hop(prev) if prev is not None else 0.0
        if lower is not None:
            rhs = rhs + lower
        step = P(rhs)
        new.append(prev - step if prev is not None else -step)
    return new


def _accumulate(ut, u):
    """ut_j += u_{i,j} for the new step (ut grows by one entry)."""
    ut = list(ut) + [np.zeros_like(u[0])]
    return [ut[j] + u[j] for j in range(len(u))]


def basis(op: Operator, P: Precond, C: np.ndarray, tau: float, k: int,
          ref: float = 0.0):
    """ut_0 .. ut_{k-1} (each d x K) from the Proposition: u_{0,0} = P_S C,
    k - 1 steps of Eq. (equ:upd), ut_j = sum_i u_{i,j}.  H = A^T A + ref I."""
    def Hop(V):
        return op.AtA(V) + ref * V

    u = [P(C)]
    ut = [u[0].copy()]
    for _ in range(1, k):
        u = recursion_step(u, P, Hop, tau)
        ut = _accumulate(ut, u)
    return ut


def compose(ut, tau: float, lam: float, ref: float = 0.0) -> np.ndarray:
    """x_k(lam) = tau sum_j (tau (lam - ref))^j ut_j (Algorithm 3 / 6)."""
    mu = tau * (lam - ref)
    x = np.zeros_like(ut[0])
    for j, v in enumerate(ut):
        x = x + mu ** j * v
    return tau * x


def ihs_iterate(op: Operator, P: Precond, C: np.ndarray, tau: float, lam: float,
                k: int) -> np.ndarray:
    """k plain IHS steps x <- x - tau P_S (A^T A x + lam x - A^T b) from 0 (Eq. (equ:ihs))."""
    x = np.zeros_like(C)
    for _ in range(k):
        x = x - tau * P(op.AtA(x) + lam * x - C)
    return x


# ------------------------------------------------------- whole path (Alg. 3)
@dataclass
class Interval:
    lo: float
    hi: float
    lam0: float
    tau: float
    rate: float
    k: int
    ref: float
    ut: list = field(default_factory=list)


def _increment(u_list, tau, lam, ref):
    mu = tau * (lam - ref)
    s = np.zeros_like(u_list[0])
    for j, v in enumerate(u_list):
        s = s + mu ** j * v
    return tau * s


def basis_adaptive(op, P, C, tau, rate, lo, hi, ref, tol, k_max):
    """The basis of ``basis`` with the step count chosen by the endpoint
    increment test.

    After step i the increment of x(lam) is tau M^i P_S A^T b; the loop stops
    once its norm times r/(1-r) is below tol * ||x(lam)|| at both interval
    ends (the worst case over the interval, per the proof of Theorem 1).
    """
    def Hop(V):
        return op.AtA(V) + ref * V

    u = [P(C)]
    ut = [u[0].copy()]
    k = 1
    for i in range(1, k_max):
        u = recursion_step(u, P, Hop, tau)
        ut = _accumulate(ut, u)
        k = i + 1
        done = True
        for lam in (lo, hi):
            inc = np.linalg.norm(_increment(u, tau, lam, ref))
            xn = np.linalg.norm(compose(ut, tau, lam, ref))
            if not (inc * rate / max(1e-300, 1.0 - rate) <= tol * xn):
                done = False
        if done:
            break
    return ut, k


def path(A, B, lambdas, SA, lam_min, lam_max, *, L=None, k=None, tol=1e-10,
         k_max=200, centred=True, taus=None, sigma_d2=0.0):
    """IHS-BIN for every lambda: returns (X[T, d, K], list of Interval).

    ``SA`` is the sketched matrix (m x d).  With ``k`` given every interval
    runs exactly k steps; otherwise the endpoint test above decides.
    ``taus`` fixes the per-interval step sizes (else the exact spectrum).
    """
    op = Operator(A)
    C = op.At(np.asarray(B).reshape(A.shape[0], -1))
    grid, lam0s = plan(lam_min, lam_max, L, sigma_d2)
    ivs = []
    for l in range(len(lam0s)):
        lo, hi, lam0 = grid[l], grid[l + 1], lam0s[l]
        P = Precond(np.asarray(SA, dtype=np.float64), lam0)
        if taus is None:
            tau, rate = step_size_from_bounds(*interval_bounds(op, P, lo, hi))
        else:
            tau, rate = float(taus[l]), 0.5
        ref = lam0 if centred else 0.0
        if k is not None:
            ut = basis(op, P, C, tau, k, ref)
            kk = k
        else:
            ut, kk = basis_adaptive(op, P, C, tau, rate, lo, hi, ref, tol, k_max)
        ivs.append(Interval(lo, hi, lam0, tau, rate, kk, ref, ut))
    lambdas = np.atleast_1d(np.asarray(lambdas, dtype=np.float64))
    X = np.empty((len(lambdas),) + C.shape)
    for t, lam in enumerate(lambdas):
        iv = ivs[interval_of(lam, grid)]
        X[t] = compose(iv.ut, iv.tau, lam, iv.ref)
    return X, ivs
