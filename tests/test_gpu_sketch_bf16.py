"""GPU parity of the Gaussian sketch on the BF16 matrix cores with the FP64
oracle of the same (BF16-rounded) sketch matrix, and of a path built on it."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, rng

pytestmark = pytest.mark.gpu


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


# ragged m, n and d; (40000, 64, 256) takes the K-split path
# (300000, 40, 96): more rows than one split may sum in FP32, so the K-splits
# are forced and added in FP64
@pytest.mark.parametrize("n,d,m", [(3000, 200, 300), (1000, 129, 77), (40000, 64, 256),
                                   (5000, 512, 1024), (257, 33, 5), (300000, 40, 96)])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_bf16_gaussian_sketch_matches_oracle(torch, ctx, n, d, m, dt):
    r = np.random.default_rng(n + d)
    A = (r.standard_normal((n, d)) * (np.arange(d) + 1.0) ** -0.5).astype(dt)
    SA = ctx.sketch_apply(dev(torch, A), "gaussian", m, seed=9, prec="bf16").cpu().numpy()
    S16 = rng.gaussian_matrix_bf16(9, m, n)
    A64 = A.astype(np.float64)
    ref = S16 @ A64
    # two BF16 terms leave at most 2^-18 |a| of each entry; FP32 sums of at
    # most 2048 exact products lose a few 2^-24 * sqrt(2048): together within
    # 2e-5 of sum |s||a| per entry
    bound = 2e-5 * (np.abs(S16) @ np.abs(A64)) + 1e-300
    err = np.abs(SA - ref)
    assert (err <= bound).all(), (err / bound).max()


@pytest.mark.parametrize("K", [1, 3])
def test_path_with_bf16_gaussian_sketch(torch, ctx, K):
    p = W.make("dense_decay_2048x256", seed=21, n=6000, d=300, K=K)
    A = np.asarray(p.A, dtype=np.float32)
    B = np.asarray(p.B, dtype=np.float32).reshape(6000, K)
    lams = W.lambda_grid(1e-3, 1e2, 40)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch="gaussian", m=300,
                            seed=4, sketch_prec=1)
    ref = direct.ridge_path(A, B, lams)
    err = direct.rel_err(X.cpu().numpy(), ref)
    assert err.max() <= 1e-6, err.max()


@pytest.mark.parametrize("m,n", [(4096, 1024), (300, 2500)])
def test_bf16_gaussian_draws_exact(torch, ctx, m, n):
    # A = I: each entry of SA is one BF16 draw times 1/sqrt(m) (a single exact
    # product in the FP32 sums), so every draw of the sketch matrix is checked
    # against BF16(FP32(z)) of the oracle's FP64 Box-Muller draw
    A = np.eye(n, dtype=np.float32)
    SA = ctx.sketch_apply(dev(torch, A), "gaussian", m, seed=13, prec="bf16").cpu().numpy()
    S16 = rng.round_bf16(rng.gaussian_draws(13, m, n))
    np.testing.assert_allclose(SA * np.sqrt(m), S16, rtol=1e-14, atol=0)
