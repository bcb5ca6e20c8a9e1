"""Seeded synthetic inputs for the ridge-path solver and for the oracle.

This module only draws data: matrices, right-hand sides and lambda grids.
It holds none of the solver's arithmetic (no sketching, no products with A
used by the method, no factorizations of the problem), so the GPU path and
the oracle can both take their inputs from here without sharing any code.

Every generator takes an integer seed and draws from NumPy's PCG64, so the
same call gives the same bytes on every machine.

Workload families (the problem is min 0.5*||A x - b||^2 + 0.5*lam*||x||^2,
Section 1, Eq. (least-square); matrix right-hand sides follow the
matrix-valued problem of Section 5.3):

* ``dense_decay``     N(0,1) entries, column j scaled by (j+1)^-alpha.
* ``dense_spectrum``  (G/sqrt(n)) diag(sigma) Q^T with G Gaussian and Q a
                      random orthogonal matrix, so the singular values are
                      sigma_i within a factor 1 +- sqrt(d/n).
* ``csr_zipf``        CSR with a fixed number of distinct columns per row,
                      drawn from a truncated Zipf law, N(0,1) values.
* ``ar1_rows``        rows N(0, Sigma^2 / sqrt(n d)) with Sigma_ij =
                      0.99^|i-j|, the random data recipe of Section 6.1.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "CsrMatrix", "Problem", "lambda_grid", "dense_decay", "dense_spectrum",
    "csr_zipf", "ar1_rows", "rhs", "make", "WORKLOADS", "serving_mix",
]


@dataclasses.dataclass
class CsrMatrix:
    """Compressed sparse rows with int32 indices, sorted columns per row."""
    n: int
    d: int
    row_ptr: np.ndarray   # int32[n+1]
    col_idx: np.ndarray   # int32[nnz]
    vals: np.ndarray      # float32/float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def shape(self):
        return (self.n, self.d)

    @property
    def dtype(self):
        return self.vals.dtype


@dataclasses.dataclass
class Problem:
    """One ridge-path instance: A (dense ndarray or CsrMatrix), B (n x K)."""
    name: str
    A: object
    B: np.ndarray
    lambdas: np.ndarray          # float64[T], the requested grid
    lam_min: float
    lam_max: float
    sketch: str                  # "gaussian" | "srht" | "countsketch" | "sjlt"
    m: int
    sketch_seed: int
    x_star: np.ndarray = None    # the planted coefficients (d x K)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def d(self):
        return self.A.shape[1]


def lambda_grid(lo: float, hi: float, T: int) -> np.ndarray:
    """T values log-spaced in [lo, hi] (both ends included), float64."""
    if T == 1:
        return np.array([lo], dtype=np.float64)
    return np.exp(np.linspace(np.log(lo), np.log(hi), T)).astype(np.float64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def dense_decay(n: int, d: int, seed: int, alpha: float = 0.7,
                dtype=np.float64) -> np.ndarray:
    """N(0,1) entries with column j multiplied by (j+1)^-alpha."""
    g = _rng(seed).standard_normal((n, d))
    g *= (np.arange(1, d + 1, dtype=np.float64) ** -alpha)[None, :]
    return np.ascontiguousarray(g.astype(dtype))


def _sigma(d: int, spectrum: str) -> np.ndarray:
    i = np.arange(d, dtype=np.float64)
    if spectrum == "exp300":
        return np.exp(-i / 300.0)
    if spectrum == "invsqrt":
        return (i + 1.0) ** -0.5
    raise ValueError(f"unknown spectrum {spectrum!r}")


def dense_spectrum(n: int, d: int, seed: int, spectrum: str = "exp300",
                   dtype=np.float32, chunk: int = 1 << 15) -> np.ndarray:
    """(G / sqrt(n)) diag(sigma) Q^T, built in row chunks.

    The right factor diag(sigma) Q^T is drawn first (Q from the QR of a
    Gaussian d x d matrix), then the Gaussian rows chunk by chunk, so peak
    host memory stays near the output size.
    """
    rng = _rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    q *= np.sign(np.diag(r))[None, :]
    right = (_sigma(d, spectrum)[:, None] * q.T) / np.sqrt(n)
    right = right.astype(np.float32) if dtype == np.float32 else right
    out = np.empty((n, d), dtype=dtype)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        g = rng.standard_normal((r1 - r0, d), dtype=np.float32 if dtype == np.float32 else np.float64)
        out[r0:r1] = (g @ right).astype(dtype)
    return out


def _zipf_cols(rng, count: int, d: int, s: float) -> np.ndarray:
    p = (np.arange(1, d + 1, dtype=np.float64)) ** -s
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(count)
    return np.minimum(np.searchsorted(cdf, u, side="right"), d - 1).astype(np.int32)


def csr_zipf(n: int, d: int, per_row: int, seed: int, s: float = 1.1,
             dtype=np.float32) -> CsrMatrix:
    """Each row holds ``per_row`` distinct columns drawn from P(j) ~ (j+1)^-s.

    Duplicate draws inside a row are redrawn until every row is distinct;
    columns are sorted inside each row; values are N(0,1).
    """
    if per_row > d:
        raise ValueError("per_row must not exceed d")
    rng = _rng(seed)
    cols = _zipf_cols(rng, n * per_row, d, s).reshape(n, per_row)
    for _ in range(10000):
        cols.sort(axis=1)
        dup = np.zeros_like(cols, dtype=bool)
        dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = _zipf_cols(rng, nd, d, s)
    else:  # pragma: no cover - the redraw loop converges in a few dozen rounds
        raise RuntimeError("could not draw distinct columns")
    vals = rng.standard_normal(n * per_row).astype(dtype)
    row_ptr = (np.arange(n + 1, dtype=np.int64) * per_row).astype(np.int32)
    return CsrMatrix(n, d, row_ptr, np.ascontiguousarray(cols.reshape(-1)), vals)


def ar1_rows(n: int, d: int, seed: int, rho: float = 0.99,
             dtype=np.float64) -> np.ndarray:
    """Rows N(0, Sigma^2 / sqrt(n d)) with Sigma_ij = rho^|i-j| (Section 6.1)."""
    rng = _rng(seed)
    idx = np.arange(d)
    sig = rho ** np.abs(idx[:, None] - idx[None, :])
    g = rng.standard_normal((n, d))
    return np.ascontiguousarray((g @ sig / (n * d) ** 0.25).astype(dtype))


def _matvec(A, X):
    """Plain A @ X for drawing the planted right-hand side."""
    if isinstance(A, CsrMatrix):
        out = np.zeros((A.n, X.shape[1]))
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
        np.add.at(out, rows, A.vals.astype(np.float64)[:, None] * X[A.col_idx])
        return out
    return A.astype(np.float64) @ X


def rhs(A, K: int, noise: float, seed: int, dtype=None, x_scale: float = 1.0):
    """B = A X* + noise * N(0,1) with X* ~ N(0, x_scale^2 I); returns (B, X*)."""
    rng = _rng(seed)
    d = A.shape[1]
    xs = x_scale * rng.standard_normal((d, K))
    B = _matvec(A, xs) + noise * rng.standard_normal((A.shape[0], K))
    dt = dtype or (A.dtype if not isinstance(A, CsrMatrix) else A.vals.dtype)
    return np.ascontiguousarray(B.astype(dt)), xs


# Named workloads.  ``scale`` shrinks n (and nnz) for tests while keeping d,
# the spectrum, the sketch and the lambda grid.
WORKLOADS = {
    "dense_decay_2048x256": dict(kind="dense_decay", n=2048, d=256, K=1, noise=0.1,
                                 dtype="f64", sketch="gaussian", m=128,
                                 lam=(1e-3, 1e2), T=50),
    "dense_exp300_131072x2048": dict(kind="dense_spectrum", spectrum="exp300", n=131072,
                                     d=2048, K=1, noise=0.05, dtype="f32", sketch="srht",
                                     m=1024, lam=(1e-4, 1e1), T=200),
    "csr_zipf_1048576x8192": dict(kind="csr_zipf", n=1 << 20, d=8192, per_row=24, K=1,
                                  noise=0.1, dtype="f32", sketch="countsketch", m=4096,
                                  lam=(1e-3, 1e2), T=100),
    "dense_invsqrt_262144x4096_k64": dict(kind="dense_spectrum", spectrum="invsqrt",
                                          n=262144, d=4096, K=64, noise=0.05, dtype="f32",
                                          sketch="gaussian", m=2048, lam=(1e-4, 1e1), T=100),
    # the random over-determined experiment of Section 6.1: AR(1) rows,
    # x* ~ N(0, I/d), noise sigma = 0.02, SJLT of sparsity 1 (CountSketch)
    "dense_ar1_20000x4000": dict(kind="ar1", n=20000, d=4000, K=1, noise=0.02, dtype="f64",
                                 sketch="countsketch", m=1600, lam=(1.0, 100.0), T=50),
    # under-determined (n < d): solved through the dual problem
    "dense_decay_8192x65536_wide": dict(kind="dense_decay", n=8192, d=65536, K=1, noise=0.1,
                                        dtype="f32", sketch="srht", m=4096,
                                        lam=(1e-2, 1e3), T=100),
}


def make(name: str, seed: int = 1000, n: int = None, d: int = None,
         K: int = None, T: int = None, m: int = None) -> Problem:
    """Build a named workload; n/d/K/T/m override the stored sizes."""
    w = dict(WORKLOADS[name])
    n = n or w["n"]
    d = d or w["d"]
    K = K or w["K"]
    T = T or w["T"]
    m = m or w["m"]
    dt = np.float64 if w["dtype"] == "f64" else np.float32
    if w["kind"] == "dense_decay":
        A = dense_decay(n, d, seed, dtype=dt)
    elif w["kind"] == "dense_spectrum":
        A = dense_spectrum(n, d, seed, w["spectrum"], dtype=dt)
    elif w["kind"] == "csr_zipf":
        A = csr_zipf(n, d, w["per_row"], seed, dtype=dt)
    elif w["kind"] == "ar1":
        A = ar1_rows(n, d, seed, dtype=dt)
    else:
        raise ValueError(w["kind"])
    xsc = d ** -0.5 if w["kind"] == "ar1" else 1.0
    B, xs = rhs(A, K, w["noise"], seed + 1, x_scale=xsc)
    lo, hi = w["lam"]
    return Problem(name, A, B, lambda_grid(lo, hi, T), lo, hi, w["sketch"], m,
                   seed + 1000, xs)


def serving_mix(count: int, seed: int = 5000, rate: float = 200.0):
    """Request stream of the serving workload: Poisson arrivals at ``rate`` per
    second (exponential gaps), n ~ U[4096, 262144], d from {128, ..., 2048},
    dense with probability 0.7 (columns scaled by (j+1)^-0.7) else CSR with 16
    entries per row, K ~ U[1, 16]; T = 100 lambdas in [1e-4, 1e1].  Returns a
    list of dicts (arrival time in seconds and the shape of each request); the
    data itself is drawn from (seed, index)."""
    r = _rng(seed)
    t = np.cumsum(r.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        out.append(dict(index=i, arrival=float(t[i]), n=int(r.integers(4096, 262145)),
                        d=int(r.choice([128, 256, 512, 1024, 2048])),
                        dense=bool(r.random() < 0.7), K=int(r.integers(1, 17)),
                        seed=seed + 1 + i))
    return out
