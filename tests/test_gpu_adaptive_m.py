"""GPU parity of the adaptive sketch-dimension search (Section 5.1,
Algorithm 4) with the FP64 oracle: the same sketches, the same decisions
(every step size and every doubling), the same scalars and iterates."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive_m, direct

pytestmark = pytest.mark.gpu

TOL_PATH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2210_12212_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def csr_dev(torch, M):
    from paper_2210_12212_amd import CsrInput
    return CsrInput(dev(torch, M.row_ptr), dev(torch, M.col_idx), dev(torch, M.vals), M.n, M.d)


def _margins_ok(ref, gamma3):
    # every doubling decision of the oracle is clear of its threshold, so
    # rounding differences cannot flip it
    return all(abs(dn / dl - gamma3) > 1e-7 for _, _, dl, dn, _ in ref.trace if dl > 0)


def _compare(res, X, trace, ref, m_cap, tol_x=1e-9):
    assert res["m"] == min(ref.m, m_cap)
    assert res["iters"] == ref.iters
    assert res["doublings"] == ref.doublings
    rt = np.array(ref.trace, dtype=np.float64).reshape(-1, 5)
    assert trace.shape == rt.shape
    np.testing.assert_array_equal(trace[:, 0], rt[:, 0])   # m per update
    np.testing.assert_array_equal(trace[:, 1], rt[:, 1])   # tau (powers of gamma1)
    np.testing.assert_array_equal(trace[:, 4], rt[:, 4])   # doublings
    np.testing.assert_allclose(trace[:, 2], rt[:, 2], rtol=1e-8)
    # delta_{k+1} shrinks far below delta_0: compare it on the scale of delta_0
    np.testing.assert_allclose(trace[:, 3], rt[:, 3], rtol=1e-6, atol=1e-12 * rt[0, 2])
    Xr = ref.X
    err = np.abs(X - Xr).max() / np.abs(Xr).max()
    assert err <= tol_x, err


CASES = [
    # kind, n, d, K, lam, m0, seed
    ("gaussian", 2000, 130, 1, 1e-2, 16, 4),
    ("srht", 4096, 200, 2, 1e-2, 8, 5),
    ("countsketch", 5000, 257, 1, 1e-1, 16, 6),
    ("sjlt", 3000, 96, 3, 1e-3, 8, 7),
]


@pytest.mark.parametrize("kind,n,d,K,lam,m0,seed", CASES)
def test_sketch_size_matches_oracle(torch, ctx, kind, n, d, K, lam, m0, seed):
    P = W.make("dense_decay_2048x256", seed=seed, n=n, d=d, K=K)
    A = np.asarray(P.A, dtype=np.float64)
    B = np.asarray(P.B, dtype=np.float64).reshape(n, K)
    s = 2 if kind == "sjlt" else 1
    m_cap = min(n, 32 * d)
    ref = adaptive_m.sketch_size(A, B, lam, kind, seed, m0, s=s, m_cap=m_cap)
    assert _margins_ok(ref, 0.5)
    res, X, tr = ctx.sketch_size(dev(torch, A), dev(torch, B), lam, sketch=kind, m=m0,
                                 seed=seed, sjlt_s=s, m_max=m_cap)
    _compare(res, X.cpu().numpy(), tr, ref, m_cap)


def test_sketch_size_float32_and_csr(torch, ctx):
    # FP32 storage is read exactly: the oracle sees the same values in FP64
    P = W.make("dense_decay_2048x256", seed=8, n=2500, d=100, K=1)
    A = np.asarray(P.A, dtype=np.float32)
    B = np.asarray(P.B, dtype=np.float32).reshape(-1, 1)
    ref = adaptive_m.sketch_size(A.astype(np.float64), B.astype(np.float64), 3e-2, "srht", 8,
                                 16, m_cap=2500)
    assert _margins_ok(ref, 0.5)
    res, X, tr = ctx.sketch_size(dev(torch, A), dev(torch, B), 3e-2, sketch="srht", m=16,
                                 seed=8, m_max=2500)
    _compare(res, X.cpu().numpy(), tr, ref, 2500)

    M = W.csr_zipf(6000, 300, 9, seed=3, dtype=np.float64)
    Bc = np.random.default_rng(2).standard_normal((6000, 2))
    ref = adaptive_m.sketch_size(M, Bc, 1.0, "countsketch", 3, 32, m_cap=6000)
    assert _margins_ok(ref, 0.5)
    res, X, tr = ctx.sketch_size(csr_dev(torch, M), dev(torch, Bc), 1.0, sketch="countsketch",
                                 m=32, seed=3, m_max=6000)
    _compare(res, X.cpu().numpy(), tr, ref, 6000)


def test_sketch_size_parameters_and_exact_hessian(torch, ctx):
    P = W.make("dense_decay_2048x256", seed=9, n=1500, d=80, K=1)
    A = np.asarray(P.A, dtype=np.float64)
    B = np.asarray(P.B, dtype=np.float64).reshape(-1, 1)
    # other gammas and eps
    kw = dict(gamma1=0.3, gamma2=0.2, gamma3=0.3, eps=1e-12, max_iter=80)
    ref = adaptive_m.sketch_size(A, B, 1e-2, "gaussian", 2, 8, m_cap=1500, **kw)
    assert _margins_ok(ref, 0.3)
    res, X, tr = ctx.sketch_size(dev(torch, A), dev(torch, B), 1e-2, sketch="gaussian", m=8,
                                 seed=2, m_max=1500, alg4=kw, trace_rows=100)
    _compare(res, X.cpu().numpy(), tr, ref, 1500)
    # m0 >= n: S = I, one Newton step reaches x*
    res, X, tr = ctx.sketch_size(dev(torch, A), dev(torch, B), 1e-2, sketch="gaussian",
                                 m=1500, seed=2, m_max=1500)
    assert res["m"] == 1500 and res["iters"] == 1 and tr[0, 1] == 1.0
    xs = direct.ridge_path(A, B, [1e-2])[0]
    np.testing.assert_allclose(X.cpu().numpy(), xs, rtol=0, atol=1e-10 * np.abs(xs).max())


def test_sketch_size_dual(torch, ctx):
    # n < d: the search runs on the dual problem (A^T with right-hand side B)
    r = np.random.default_rng(4)
    A = r.standard_normal((120, 700)) * (np.arange(700) + 1.0) ** -0.6
    B = r.standard_normal((120, 1))
    ref = adaptive_m.sketch_size(A, B, 1e-2, "srht", 6, 8, dual=True, m_cap=700)
    assert _margins_ok(ref, 0.5)
    res, Z, tr = ctx.sketch_size(dev(torch, A), dev(torch, B), 1e-2, sketch="srht", m=8, seed=6,
                                 m_max=700)
    assert Z.shape == (120, 1)
    _compare(res, Z.cpu().numpy(), tr, ref, 700)


def test_sketch_size_errors(torch, ctx):
    from paper_2210_12212_amd import IhsbinError
    A = dev(torch, np.random.default_rng(0).standard_normal((200, 20)))
    B = dev(torch, np.ones((200, 1)))
    with pytest.raises(IhsbinError):
        ctx.sketch_size(A, B, 1e-2, alg4=dict(gamma1=1.5))
    with pytest.raises(IhsbinError):
        ctx.sketch_size(A, B, 0.0)
    with pytest.raises(IhsbinError):
        ctx.sketch_size(A, B, 1e-2, alg4=dict(max_armijo=0))


@pytest.mark.parametrize("kind", ["srht", "countsketch", "gaussian"])
def test_path_with_algorithm4_sizing(torch, ctx, kind):
    # adaptive_m = 2: the build sizes m by Algorithm 4 at lam_min and keeps
    # that sketch; the path meets the per-lambda bar and m_used equals the
    # standalone search's m
    P = W.make("dense_decay_2048x256", seed=12, n=4096, d=160, K=2)
    A = np.asarray(P.A, dtype=np.float64)
    B = np.asarray(P.B, dtype=np.float64).reshape(4096, 2)
    lams = W.lambda_grid(1e-2, 1e2, 30)
    Ad, Bd = dev(torch, A), dev(torch, B)
    X, rep = ctx.solve_path(Ad, Bd, lams, sketch=kind, seed=3, adaptive_m=2, m=16)
    ref = direct.ridge_path(A, B, lams)
    err = direct.rel_err(X.cpu().numpy(), ref)
    assert err.max() <= TOL_PATH, err.max()
    res, _, _ = ctx.sketch_size(Ad, Bd, 1e-2, sketch=kind, seed=3, m=16)
    assert rep["m_used"] >= res["m"]
