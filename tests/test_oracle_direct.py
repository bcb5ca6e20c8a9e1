"""Pins for the graded reference (oracle.direct): checked against closed
forms, brute force and invariants, never against itself."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import direct


def _svd_path(A, b, lambdas):
    # Section 2.1: x*(lam) = V (Sigma^2 + lam I)^-1 Sigma U^T b
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    Utb = U.T @ b
    return np.stack([Vt.T @ ((s / (s * s + lam))[:, None] * Utb) for lam in lambdas])


@pytest.fixture(scope="module")
def small():
    A = W.dense_decay(512, 64, seed=7)
    B, _ = W.rhs(A, 3, 0.1, seed=8)
    lams = W.lambda_grid(1e-3, 1e2, 9)
    return A, B, lams


def test_matches_svd_closed_form(small):
    A, B, lams = small
    X = direct.ridge_path(A, B, lams)
    Xs = _svd_path(A, B, lams)
    assert direct.rel_err(X, Xs).max() < 1e-10


def test_kkt_residual_with_A_directly(small):
    A, B, lams = small
    X = direct.ridge_path(A, B, lams)
    AtB = A.T @ B
    for t, lam in enumerate(lams):
        r = A.T @ (A @ X[t] - B) + lam * X[t]
        assert np.linalg.norm(r) / np.linalg.norm(AtB) < 1e-12


def test_large_lambda_limit(small):
    A, B, _ = small
    G = A.T @ A
    g2 = np.linalg.norm(G, 2)
    lam = 1e6 * g2
    x = direct.ridge_path(A, B, [lam])[0]
    c = A.T @ B
    # lam x - c = -G (G + lam I)^-1 c, so its norm is at most ||G|| / lam ||c||
    assert np.linalg.norm(lam * x - c) / np.linalg.norm(c) <= g2 / lam * 1.0000001


def test_one_column_closed_form():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((40, 1))
    b = rng.standard_normal((40, 1))
    for lam in (1e-3, 0.5, 7.0):
        x = direct.ridge_path(a, b, [lam])[0, 0, 0]
        assert x == pytest.approx(float(a[:, 0] @ b[:, 0]) / (float(a[:, 0] @ a[:, 0]) + lam), rel=1e-13)


def test_two_columns_exact_cramer():
    # brute force in exact rationals: (A^T A + lam I) x = A^T b by Cramer's rule
    A = [[1, 2], [3, -1], [0, 4], [2, 2]]
    b = [3, -2, 5, 1]
    for lam in (Fraction(1, 3), Fraction(2), Fraction(1, 1000)):
        g11 = sum(r[0] * r[0] for r in A) + lam
        g12 = sum(r[0] * r[1] for r in A)
        g22 = sum(r[1] * r[1] for r in A) + lam
        c1 = sum(r[0] * v for r, v in zip(A, b))
        c2 = sum(r[1] * v for r, v in zip(A, b))
        det = g11 * g22 - g12 * g12
        exact = [(c1 * g22 - g12 * c2) / det, (g11 * c2 - g12 * c1) / det]
        x = direct.ridge_path(np.array(A, float), np.array(b, float)[:, None], [float(lam)])[0, :, 0]
        for xi, ei in zip(x, exact):
            assert xi == pytest.approx(float(ei), rel=1e-13)


def test_orthonormal_columns():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((300, 20)))
    b = rng.standard_normal((300, 2))
    for lam in (1e-4, 1.0, 30.0):
        x = direct.ridge_path(Q, b, [lam])[0]
        np.testing.assert_allclose(x, Q.T @ b / (1.0 + lam), rtol=1e-12, atol=1e-14)


def test_monotone_in_lambda(small):
    A, B, _ = small
    lams = W.lambda_grid(1e-4, 1e3, 40)
    X = direct.ridge_path(A, B[:, :1], lams)
    norms = np.linalg.norm(X[:, :, 0], axis=1)
    assert np.all(np.diff(norms) < 0)
    # training loss of Section 6.1 increases with lambda along the exact path
    Ltr = [0.5 * np.sum((A @ X[t] - B[:, :1]) ** 2) + 0.5 * lam * np.sum(X[t] ** 2)
           for t, lam in enumerate(lams)]
    assert np.all(np.diff(Ltr) > 0)


def test_csr_matches_dense():
    Ac = W.csr_zipf(500, 40, 6, seed=11)
    Ad = np.zeros((500, 40))
    rows = np.repeat(np.arange(500), 6)
    Ad[rows, Ac.col_idx] = Ac.vals
    B, _ = W.rhs(Ad, 1, 0.1, seed=12)
    lams = [1e-3, 1.0, 100.0]
    np.testing.assert_allclose(direct.ridge_path(Ac, B, lams), _svd_path(Ad, B, lams),
                               rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_dual_form_for_wide_matrices(dt):
    # n < d: the dual form A^T (A A^T + lam I)^-1 b (Section 5.2) against the
    # SVD closed form of Section 2.1 (the d x d primal Gram is rank n here) and
    # the KKT residual computed with A
    A = W.dense_decay(60, 240, seed=17, dtype=dt)
    B, _ = W.rhs(A, 2, 0.1, seed=18)
    lams = W.lambda_grid(1e-3, 1e2, 7)
    X = direct.ridge_path_dual(A, B, lams)
    A64 = np.asarray(A, dtype=np.float64)
    assert direct.rel_err(X, _svd_path(A64, B, lams)).max() < 1e-10
    assert direct.rel_err(X, direct.ridge_path(A, B, lams)).max() < 1e-9
    AtB = A64.T @ B
    for t, lam in enumerate(lams):
        r = A64.T @ (A64 @ X[t] - B) + lam * X[t]
        assert np.linalg.norm(r) / np.linalg.norm(AtB) < 1e-11


# ---- the per-lambda error metric every parity test reads
def test_rel_err_hand_computed():
    # two lambdas, d = 2, K = 1: block 0 off by 0.5 in a vector of norm 5,
    # block 1 exact
    ref = np.array([[[3.0], [4.0]], [[1.0], [0.0]]])
    got = np.array([[[3.0], [4.5]], [[1.0], [0.0]]])
    e = direct.rel_err(got, ref)
    assert e.shape == (2,)
    assert e[0] == pytest.approx(0.1, rel=1e-15)
    assert e[1] == 0.0


def test_rel_err_reports_large_errors():
    rng = np.random.default_rng(11)
    ref = rng.standard_normal((4, 5, 3))
    assert np.allclose(direct.rel_err(-ref, ref), 2.0, rtol=1e-14)
    assert np.allclose(direct.rel_err(np.zeros_like(ref), ref), 1.0, rtol=1e-14)
    assert np.allclose(direct.rel_err(3.0 * ref, ref), 2.0, rtol=1e-14)
    # a NaN anywhere in a block is never reported as a small error
    bad = ref.copy()
    bad[2, 1, 0] = np.nan
    e = direct.rel_err(bad, ref)
    assert not (e[2] <= 1.0)
    assert np.all(e[[0, 1, 3]] == 0.0)


def test_rel_err_is_per_lambda_frobenius():
    # the norm runs over the whole d x K block of one lambda (all right-hand
    # sides together), and blocks do not mix
    ref = np.zeros((3, 2, 2))
    ref[:, 0, 0] = 1.0
    ref[:, 1, 1] = 1.0          # every block has Frobenius norm sqrt(2)
    got = ref.copy()
    got[1, 0, 1] = 1.0          # only block 1 is wrong, by norm 1
    got[2, 1, 0] = 2.0          # block 2 is wrong by norm 2
    e = direct.rel_err(got, ref)
    assert e[0] == 0.0
    assert e[1] == pytest.approx(1.0 / np.sqrt(2.0), rel=1e-15)
    assert e[2] == pytest.approx(2.0 / np.sqrt(2.0), rel=1e-15)


def test_rel_err_rejects_mismatched_sizes():
    with pytest.raises(ValueError):
        direct.rel_err(np.zeros((2, 3, 1)), np.ones((2, 4, 1)))


# ---- the eigendecomposition form used for many lambdas at large d
def test_eig_form_matches_cholesky_and_svd(small):
    A, B, lams = small
    X = direct.ridge_path_eig(A, B, lams)
    assert direct.rel_err(X, direct.ridge_path(A, B, lams)).max() < 1e-10
    assert direct.rel_err(X, _svd_path(A, B, lams)).max() < 1e-10


def test_eig_form_csr_matches_cholesky():
    A = W.csr_zipf(3000, 96, 6, seed=21)
    B, _ = W.rhs(A, 2, 0.1, seed=22)
    lams = W.lambda_grid(1e-3, 1e2, 7)
    X = direct.ridge_path_eig(A, B, lams)
    assert direct.rel_err(X, direct.ridge_path(A, B, lams)).max() < 1e-10
