"""Pins of the Algorithm 4 oracle (Section 5.1) against facts that do not
come from the oracle itself: the ridge solution by a direct solve, the
closed form of f on a line (f is quadratic), and the exact-Hessian case in
which the direction is the Newton step."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive_m, direct


def _problem(n=512, d=48, K=1, seed=3):
    P = W.make("dense_decay_2048x256", seed=seed, n=n, d=d, K=K)
    return np.asarray(P.A, dtype=np.float64), np.asarray(P.B, dtype=np.float64)


def _f(A, B, lam, X):
    R = A @ X - B
    return 0.5 * np.sum(R * R) + 0.5 * lam * np.sum(X * X)


def test_exact_hessian_takes_one_newton_step():
    # m >= n means S = I: D_0 = H^-1 grad f(0) = -x*, delta_0 = 2 (f(0) - f*),
    # the full step passes the Armijo test and lands on x*
    A, B = _problem(n=300, d=40, K=2)
    lam = 0.3
    xs = direct.ridge_path(A, B, [lam])[0]
    r = adaptive_m.sketch_size(A, B, lam, "gaussian", 1, m0=300)
    assert r.iters == 1 and r.doublings == 0 and r.m == 300
    m, tau, delta0, delta1, doubled = r.trace[0]
    assert tau == 1.0 and doubled == 0
    f0 = _f(A, B, lam, np.zeros_like(xs))
    fs = _f(A, B, lam, xs)
    assert delta0 == pytest.approx(2.0 * (f0 - fs), rel=1e-10)
    assert abs(delta1) <= 1e-20 * delta0 + 1e-300 or delta1 <= 1e-12 * delta0
    np.testing.assert_allclose(r.X, xs, rtol=0, atol=1e-10 * np.abs(xs).max())


@pytest.mark.parametrize("kind", ["gaussian", "countsketch", "srht", "sjlt"])
def test_iterates_reach_the_ridge_solution(kind):
    # a sketched direction with a tight stop test still ends at x*(lam)
    A, B = _problem(n=1024, d=64, K=1)
    lam = 0.05
    xs = direct.ridge_path(A, B, [lam])[0]
    r = adaptive_m.sketch_size(A, B, lam, kind, 11, m0=8, s=2 if kind == "sjlt" else 1,
                               eps=1e-24, max_iter=400)
    err = np.linalg.norm(r.X - xs) / np.linalg.norm(xs)
    assert err <= 1e-8, err


def test_armijo_steps_are_the_largest_accepted():
    # along X_k - tau D_k, f is quadratic: f(X - tau D) - f(X) =
    # -tau <D, g> + tau^2/2 <D, (A^T A + lam I) D>; every accepted tau passes
    # Eq. (armijo) and tau / gamma1 (when tau < 1) does not
    A, B = _problem(n=800, d=96, K=2)
    lam, g1, g2 = 1e-2, 0.5, 1e-4
    r = adaptive_m.sketch_size(A, B, lam, "countsketch", 5, m0=16, keep_iterates=True,
                               gamma1=g1, gamma2=g2)
    assert r.iters >= 3
    H = A.T @ A + lam * np.eye(A.shape[1])
    C = A.T @ B
    for k, (m, tau, delta, _, _) in enumerate(r.trace):
        X0, X1 = r.iterates[k], r.iterates[k + 1]
        D = (X0 - X1) / tau
        g = H @ X0 - C
        assert np.sum(D * g) == pytest.approx(delta, rel=1e-9)
        q = np.sum(D * (H @ D))

        def decrease(t):
            return -t * delta + 0.5 * t * t * q

        assert decrease(tau) <= -g2 * tau * delta * (1 - 1e-9)
        if tau < 1.0:
            assert decrease(tau / g1) > -g2 * (tau / g1) * delta
    # f never increases
    fs = [_f(A, B, lam, X) for X in r.iterates]
    assert all(b <= a * (1 + 1e-14) for a, b in zip(fs, fs[1:]))


def test_m_doubles_exactly_when_progress_stalls():
    A, B = _problem(n=2048, d=128, K=1)
    lam, g3 = 1e-3, 0.5
    r = adaptive_m.sketch_size(A, B, lam, "srht", 9, m0=8, gamma3=g3, m_cap=2048)
    assert r.doublings >= 2 and r.m > 8
    m_prev = 8
    for m, tau, delta, delta_next, doubled in r.trace:
        assert m == m_prev
        stalled = delta_next >= g3 * delta
        assert doubled == (1 if (stalled and m < 2048) else 0)
        m_prev = min(2 * m, 2048) if doubled else m
    assert r.m == m_prev
    # the search stops by its test
    assert r.trace[-1][3] <= 1e-8 * r.trace[0][2] or r.iters == 50


def test_scale_invariance():
    # B -> c B scales X by c and delta by c^2; the decisions do not change
    A, B = _problem(n=600, d=50, K=1)
    r1 = adaptive_m.sketch_size(A, B, 0.1, "countsketch", 2, m0=8)
    r2 = adaptive_m.sketch_size(A, 8.0 * B, 0.1, "countsketch", 2, m0=8)
    assert r1.m == r2.m and r1.iters == r2.iters
    assert [t[1] for t in r1.trace] == [t[1] for t in r2.trace]
    np.testing.assert_allclose(8.0 * r1.X, r2.X, rtol=1e-9, atol=1e-12)


def test_dual_form_reaches_the_ridge_solution():
    # n < d: the search on Eq. (ls_reg:d) ends at z with A^T z = x*(lam),
    # checked against the primal direct solve
    r = np.random.default_rng(4)
    A = r.standard_normal((60, 150)) * (np.arange(150) + 1.0) ** -0.6
    B = r.standard_normal((60, 2))
    lam = 1e-2
    res = adaptive_m.sketch_size(A, B, lam, "countsketch", 6, 4, dual=True, eps=1e-26,
                                 max_iter=400)
    xs = direct.ridge_path(A, B, [lam])[0]
    np.testing.assert_allclose(A.T @ res.X, xs, rtol=0, atol=1e-9 * np.abs(xs).max())
