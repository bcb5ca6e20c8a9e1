"""GPU parity of the Gaussian sketch on the FP8 matrix cores with the FP64
oracle of the same e4m3 sketch matrix and e4m3 form of A, and of a path built
on it."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, rng, sketch

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


# ragged m, n and d; (40000, 64, 256) takes the K-split path; column scales
# from 1e-6 to 1e5, one zero column
# (300000, 40, 96): more rows than one split may sum in FP32, so the K-splits
# are forced and added in FP64
@pytest.mark.parametrize("n,d,m", [(3000, 200, 300), (1000, 129, 77), (40000, 64, 256),
                                   (5000, 512, 1024), (257, 33, 5), (300000, 40, 96)])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_fp8_gaussian_sketch_matches_oracle(torch, ctx, n, d, m, dt):
    r = np.random.default_rng(n + d)
    A = r.standard_normal((n, d)) * (np.arange(d) + 1.0) ** -0.5
    A *= 10.0 ** r.integers(-6, 6, d)
    A[:, d // 2] = 0.0
    A = A.astype(dt)
    SA = ctx.sketch_apply(dev(torch, A), "gaussian", m, seed=9, prec="fp8").cpu().numpy()
    S8 = rng.gaussian_matrix_fp8(9, m, n)
    At = sketch.fp8_reconstruct(A.astype(np.float64))
    ref = S8 @ At
    # the e4m3 products are exact in FP32; FP32 sums of at most 2048 rows and
    # FP32 sums of at most 128 of those lose within 2e-5 of sum |s||a~|
    bound = 2e-5 * (np.abs(S8) @ np.abs(At)) + 1e-300
    err = np.abs(SA - ref)
    assert (err <= bound).all(), (err / bound).max()


@pytest.mark.parametrize("m,n", [(4096, 1024), (300, 2500)])
def test_fp8_gaussian_draws_exact(torch, ctx, m, n):
    # A = I (its e4m3 form is exact): each entry of SA is one e4m3 draw times
    # 1/sqrt(m), checked against E4M3(FP32(z)) of the oracle's FP64 draw
    A = np.eye(n, dtype=np.float32)
    SA = ctx.sketch_apply(dev(torch, A), "gaussian", m, seed=13, prec="fp8").cpu().numpy()
    S8 = rng.round_e4m3(rng.gaussian_draws(13, m, n))
    np.testing.assert_allclose(SA * np.sqrt(m), S8, rtol=1e-14, atol=0)


@pytest.mark.parametrize("K", [1, 3])
def test_path_with_fp8_gaussian_sketch(torch, ctx, K):
    p = W.make("dense_decay_2048x256", seed=21, n=6000, d=300, K=K)
    A = np.asarray(p.A, dtype=np.float32)
    B = np.asarray(p.B, dtype=np.float32).reshape(6000, K)
    lams = W.lambda_grid(1e-3, 1e2, 40)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch="gaussian", m=300,
                            seed=4, sketch_prec=2)
    ref = direct.ridge_path(A, B, lams)
    err = direct.rel_err(X.cpu().numpy(), ref)
    assert err.max() <= 1e-6, err.max()


def test_fp8_rejected_for_csr(torch, ctx):
    from paper_2210_12212_amd import CsrInput, IhsbinError
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda:0")
    ci = torch.tensor([0, 1], dtype=torch.int32, device="cuda:0")
    v = torch.tensor([1.0, 2.0], dtype=torch.float64, device="cuda:0")
    with pytest.raises(IhsbinError):
        ctx.sketch_apply(CsrInput(rp, ci, v, 2, 2), "gaussian", 4, seed=1, prec="fp8")
