"""Pins for the step-by-step IHS-BIN oracle (oracle.ihs_bin)."""
from math import comb

import numpy as np
import pytest

import workloads as W
from oracle import direct, ihs_bin, sketch


@pytest.fixture(scope="module")
def prob():
    A = W.dense_decay(400, 24, seed=21)
    B, _ = W.rhs(A, 2, 0.1, seed=22)
    SA = sketch.apply("gaussian", A, 5, 96)
    return A, B, SA


def test_plan_natural_log_and_boundaries():
    grid, lam0 = ihs_bin.plan(1e-4, 1e1)
    assert len(grid) == 24                          # L = floor(2 ln 1e5) = 23
    assert grid[0] == 1e-4 and grid[-1] == 1e1
    np.testing.assert_allclose(lam0, np.sqrt(grid[:-1] * grid[1:]))
    np.testing.assert_allclose(grid[1:] / grid[:-1], (1e5) ** (1 / 23))
    assert ihs_bin.interval_of(grid[3], grid) == 2  # a boundary goes to the lower interval
    assert ihs_bin.interval_of(1e-4, grid) == 0
    assert ihs_bin.interval_of(1e1, grid) == 22
    assert ihs_bin.num_intervals(1.0, 1.0) == 1


@pytest.mark.parametrize("centred", [False, True])
def test_proposition_equals_plain_ihs(prob, centred):
    # P1: the basis composition equals k plain IHS steps from x0 = 0, any lambda
    A, B, SA = prob
    op = ihs_bin.Operator(A)
    C = op.At(B)
    lam0 = 0.3
    P = ihs_bin.Precond(SA, lam0)
    tau, k = 0.7, 9
    ref = lam0 if centred else 0.0
    ut = ihs_bin.basis(op, P, C, tau, k, ref)
    for lam in (0.05, 0.2, lam0, 0.45, 2.0):
        x_basis = ihs_bin.compose(ut, tau, lam, ref)
        x_plain = ihs_bin.ihs_iterate(op, P, C, tau, lam, k)
        assert np.linalg.norm(x_basis - x_plain) <= 1e-11 * np.linalg.norm(x_plain)


def test_identity_preconditioner_is_gd_bin(prob):
    # P2: with P_S := I and ref 0 the basis is Section 3's GD-BIN basis,
    # u_j = sum_{i=0}^{k-1-j} C(i+j, j) (I - tau A^T A)^i A^T b, up to (-1)^j.
    A, B, _ = prob
    op = ihs_bin.Operator(A)
    c = op.At(B[:, :1])
    G = A.T @ A
    tau = 1.0 / np.linalg.norm(G, 2)
    k = 7
    ut = ihs_bin.basis(op, lambda v: v, c, tau, k, 0.0)
    N = np.eye(G.shape[0]) - tau * G
    powers = [np.linalg.matrix_power(N, i) for i in range(k)]
    for j in range(k):
        u_gd = sum(comb(i + j, j) * powers[i] @ c for i in range(k - j))
        np.testing.assert_allclose((-1) ** j * ut[j], u_gd, rtol=1e-10, atol=1e-12 * np.abs(u_gd).max())
    # and Algorithm 1's composition uses (-tau lam)^j
    lam = 0.2
    x_gd = tau * sum((-tau * lam) ** j * sum(comb(i + j, j) * powers[i] @ c for i in range(k - j))
                     for j in range(k))
    np.testing.assert_allclose(ihs_bin.compose(ut, tau, lam, 0.0), x_gd, rtol=1e-10)


def test_commuting_case_closed_form(prob):
    # P3: S = I_n makes P_S = (A^T A + lam0 I)^-1 commute with A^T A; per
    # eigen-direction u_{i,j} = C(i,j) N^(i-j) (-p)^j p a.
    A, B, _ = prob
    op = ihs_bin.Operator(A)
    c = op.At(B[:, :1])[:, 0]
    lam0, tau, k = 0.5, 0.9, 8
    P = ihs_bin.Precond(np.asarray(A, float), lam0)
    h, V = np.linalg.eigh(A.T @ A)
    a = V.T @ c
    p = 1.0 / (h + lam0)
    for ref in (0.0, lam0):
        ut = ihs_bin.basis(op, P, c[:, None], tau, k, ref)
        Nd = 1.0 - tau * p * (h + ref)
        for j in range(k):
            want = sum(comb(i, j) * Nd ** (i - j) * (-p) ** j * p * a for i in range(j, k))
            np.testing.assert_allclose(V.T @ ut[j][:, 0], want, rtol=1e-9,
                                       atol=1e-11 * np.abs(want).max())


def test_theorem1_rate_bound():
    # P4: with rho1, rho2 the exact extreme eigenvalues of C_S and
    # alpha = 2 sqrt(rho1 rho2) / (sqrt(kt) + 1/sqrt(kt)), every step of IHS with
    # lam0 = sqrt(lmin lmax) contracts delta_k by ((kt - 1)/(kt + 1))^2.
    A = W.dense_decay(300, 12, seed=31)
    B, _ = W.rhs(A, 1, 0.1, seed=32)
    n, d = A.shape
    lmin, lmax = 0.05, 0.5
    lam0 = np.sqrt(lmin * lmax)
    SA = sketch.apply("gaussian", A, 9, 60)
    S = None
    from oracle import rng as orng
    S = orng.gaussian_matrix(9, 60, n)
    Abar = np.vstack([A, np.sqrt(lam0) * np.eye(d)])
    Ubar, _, _ = np.linalg.svd(Abar, full_matrices=False)
    Sbar = np.block([[S, np.zeros((60, d))], [np.zeros((d, n)), np.eye(d)]])
    CS = (Sbar @ Ubar).T @ (Sbar @ Ubar)
    ev = np.linalg.eigvalsh(CS)
    rho1, rho2 = ev[-1], ev[0]
    kt = rho1 * lmax / (rho2 * lmin)
    alpha = 2 * np.sqrt(rho1 * rho2) / (np.sqrt(kt) + 1 / np.sqrt(kt))
    # the step-size rule used by the solver gives the same alpha from mu = 1/rho
    tau, rate = ihs_bin.step_size(1 / rho1, 1 / rho2, lmin, lmax, lam0)
    assert tau == pytest.approx(alpha, rel=1e-12)
    assert rate == pytest.approx((kt - 1) / (kt + 1), rel=1e-12)
    op = ihs_bin.Operator(A)
    P = ihs_bin.Precond(SA, lam0)
    C = op.At(B)
    bound = ((kt - 1) / (kt + 1)) ** 2
    for lam in (lmin, 0.11, lam0, 0.3, lmax):
        xs = direct.ridge_path(A, B, [lam])[0]
        At = np.vstack([A, np.sqrt(lam) * np.eye(d)])
        x = np.zeros_like(C)
        delta = 0.5 * np.sum((At @ (x - xs)) ** 2)
        for _ in range(12):
            x = x - alpha * P(op.AtA(x) + lam * x - C)
            dn = 0.5 * np.sum((At @ (x - xs)) ** 2)
            assert dn <= bound * delta * (1 + 1e-9) + 1e-300
            delta = dn


def test_spectrum_inclusion_for_every_lambda(prob):
    # the spectrum of P_S (A^T A + lam I) lies in [mu_min min(1, lam/lam0), mu_max max(1, lam/lam0)]
    A, _, SA = prob
    op = ihs_bin.Operator(A)
    lam0 = 0.2
    P = ihs_bin.Precond(SA, lam0)
    mu_min, mu_max = ihs_bin.spectrum_bounds(op, P)
    G = A.T @ A
    Pm = P(np.eye(G.shape[0]))
    for lam in (0.01, 0.1, 0.2, 0.5, 3.0):
        ev = np.sort(np.linalg.eigvals(Pm @ (G + lam * np.eye(len(G)))).real)
        assert ev[0] >= mu_min * min(1, lam / lam0) * (1 - 1e-9)
        assert ev[-1] <= mu_max * max(1, lam / lam0) * (1 + 1e-9)


def test_interval_bounds_hold_for_every_lambda(prob):
    # c_min = lambda_min at lo and c_max = lambda_max at hi bound the spectrum
    # for every lam in [lo, hi], are attained at the ends, and sit inside the
    # looser [mu_min lo/lam0, mu_max hi/lam0] built from the spectrum at lam0
    A, _, SA = prob
    op = ihs_bin.Operator(A)
    lo, hi = 0.05, 0.8
    lam0 = np.sqrt(lo * hi)
    P = ihs_bin.Precond(SA, lam0)
    cmin, cmax = ihs_bin.interval_bounds(op, P, lo, hi)
    G = A.T @ A
    Pm = P(np.eye(G.shape[0]))
    lows, highs = [], []
    for lam in np.linspace(lo, hi, 9):
        ev = np.sort(np.linalg.eigvals(Pm @ (G + lam * np.eye(len(G)))).real)
        assert ev[0] >= cmin * (1 - 1e-9) and ev[-1] <= cmax * (1 + 1e-9)
        lows.append(ev[0])
        highs.append(ev[-1])
    assert np.all(np.diff(lows) >= -1e-12) and np.all(np.diff(highs) >= -1e-12)
    assert lows[0] == pytest.approx(cmin, rel=1e-9) and highs[-1] == pytest.approx(cmax, rel=1e-9)
    mu_min, mu_max = ihs_bin.spectrum_bounds(op, P)
    assert cmin >= mu_min * lo / lam0 * (1 - 1e-12) and cmax <= mu_max * hi / lam0 * (1 + 1e-12)
    tau, rate = ihs_bin.step_size_from_bounds(cmin, cmax)
    assert max(abs(1 - tau * cmin), abs(1 - tau * cmax)) == pytest.approx(rate, rel=1e-12)


def test_centred_and_printed_expansions_agree(prob):
    A, B, SA = prob
    lams = W.lambda_grid(1e-3, 1e2, 13)
    X0, iv0 = ihs_bin.path(A, B, lams, SA, 1e-3, 1e2, k=6, centred=False)
    X1, iv1 = ihs_bin.path(A, B, lams, SA, 1e-3, 1e2, k=6, centred=True,
                           taus=[iv.tau for iv in iv0])
    assert direct.rel_err(X1, X0).max() < 1e-10


@pytest.mark.parametrize("kind", ["gaussian", "srht", "countsketch"])
def test_converged_path_matches_direct(kind):
    # P5: the adaptive oracle reaches the exact path
    A = W.dense_decay(600, 32, seed=41)
    B, _ = W.rhs(A, 2, 0.1, seed=42)
    lams = W.lambda_grid(1e-3, 1e2, 17)
    SA = sketch.apply(kind, A, 6, 256)
    X, ivs = ihs_bin.path(A, B, lams, SA, 1e-3, 1e2, tol=1e-11)
    assert direct.rel_err(X, direct.ridge_path(A, B, lams)).max() < 1e-8
    assert all(iv.rate < 1 for iv in ivs)


def test_matrix_rhs_is_columnwise(prob):
    # Algorithm 5 is Algorithm 2 applied to each column of B
    A, B, SA = prob
    lams = [0.01, 0.5, 10.0]
    X, ivs = ihs_bin.path(A, B, lams, SA, 1e-3, 1e2, k=5)
    taus = [iv.tau for iv in ivs]
    for col in range(B.shape[1]):
        Xc, _ = ihs_bin.path(A, B[:, col:col + 1], lams, SA, 1e-3, 1e2, k=5, taus=taus)
        # identical in exact arithmetic; BLAS rounds a K-column product and a
        # one-column product differently, so the tolerance follows the scale of X
        np.testing.assert_allclose(X[:, :, col:col + 1], Xc, rtol=1e-12,
                                   atol=1e-13 * np.abs(X).max())


def test_refined_centres_remark():
    # the remark after Theorem 1: (lam0 + s)^2 = (lo + s)(hi + s); s = 0 is the
    # geometric centre, s -> infinity the arithmetic one
    grid, c0 = ihs_bin.plan(1e-3, 1e2, 9)
    np.testing.assert_allclose(c0, np.sqrt(grid[:-1] * grid[1:]), rtol=1e-14)
    for s in (1e-3, 0.7, 50.0):
        g, c = ihs_bin.plan(1e-3, 1e2, 9, sigma_d2=s)
        np.testing.assert_array_equal(g, grid)
        np.testing.assert_allclose((c + s) ** 2, (g[:-1] + s) * (g[1:] + s), rtol=1e-13)
        assert (c >= g[:-1]).all() and (c <= g[1:]).all()
    g, c = ihs_bin.plan(1e-3, 1e2, 9, sigma_d2=1e9)
    np.testing.assert_allclose(c, 0.5 * (g[:-1] + g[1:]), rtol=1e-6)


def test_refined_centres_lower_the_exact_rate():
    # with the exact Hessian (S = I) the spectrum of P (A^T A + lam I) over an
    # interval is {(s_i + lam) / (s_i + lam0)}: with sigma_d^2 comparable to
    # the lambdas the refined centre gives a smaller worst-case rate
    r = np.random.default_rng(4)
    n, d = 400, 30
    U, _ = np.linalg.qr(r.standard_normal((n, d)))
    sig2 = np.geomspace(0.5, 50.0, d)
    A = U * np.sqrt(sig2)
    op = ihs_bin.Operator(A)
    s = float(np.linalg.eigvalsh(A.T @ A)[0])
    g, c_plain = ihs_bin.plan(1e-2, 1e2, 4)
    _, c_ref = ihs_bin.plan(1e-2, 1e2, 4, sigma_d2=s)
    for l in range(4):
        rates = []
        for c in (c_plain[l], c_ref[l]):
            P = ihs_bin.Precond(A, c)
            rates.append(ihs_bin.step_size_from_bounds(*ihs_bin.interval_bounds(op, P, g[l], g[l + 1]))[1])
        assert rates[1] <= rates[0] + 1e-12, (l, rates)
        # closed form: the extremes sit at sigma^2 = s, c in [1/k, k] with
        # k^2 = (hi + s) / (lo + s), so the rate is (k^2 - 1) / (k^2 + 1)
        k2 = (g[l + 1] + s) / (g[l] + s)
        assert rates[1] == pytest.approx((k2 - 1) / (k2 + 1), rel=1e-9)
