"""GPU checks of the basis products on the FP32 matrix cores (precision
variants of the recursion, which refines x with every step: Section 4, the
fixed point does not depend on how P_S was formed, only the products' error
limits what is reached).

* ``ata_apply_f32`` is not an ABI call: the FP32 products are reached
  through builds with basis_prec; their accuracy is checked on the path.
* IHSBIN_BASIS_F32: every step in FP32, error reported per lambda against the
  FP64 oracle, within the 1e-4 the precision variant is specified to.
* IHSBIN_BASIS_MIXED: FP64 until the increments are small, then FP32; the
  path stays within 1e-6 of the oracle at every lambda.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct

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


@pytest.fixture(scope="module")
def problem():
    p = W.make("dense_exp300_131072x2048", n=32768, d=512, T=60)
    ev, V = direct.eig_of_gram(direct.gram(p.A))
    ref = direct.solve_from_eig(ev, V, direct.atb(p.A, p.B), p.lambdas)
    return p, ref


@pytest.mark.parametrize("K", [1, 5])
def test_fp32_products_every_step(torch, ctx, problem, K):
    p, ref = problem
    B = p.B if K == 1 else np.ascontiguousarray(np.repeat(p.B, K, axis=1) *
                                                np.linspace(1.0, 2.0, K)[None, :]).astype(np.float32)
    refK = ref if K == 1 else direct.solve_from_eig(
        *direct.eig_of_gram(direct.gram(p.A)), direct.atb(p.A, B), p.lambdas)
    X, rep = ctx.solve_path(dev(torch, p.A), dev(torch, B), p.lambdas, sketch="srht", m=1024,
                            seed=3, tol=1e-7, basis_prec=1, timing=1, k_max=40)
    err = direct.rel_err(X.cpu().numpy(), refK)
    print(f"FP32 products: max rel err {err.max():.3e}, k_max {rep['k_max_used']}, "
          f"launches f32 {rep['ata_f32_launches']} f64 {rep['ata_launches']}")
    assert rep["ata_f32_launches"] > 0 and rep["ata_launches"] == 0
    assert err.max() <= 1e-4, err


@pytest.mark.parametrize("switch", [1e-3, 1e-2])
def test_mixed_products_keep_1e6(torch, ctx, problem, switch):
    p, ref = problem
    X64, rep64 = ctx.solve_path(dev(torch, p.A), dev(torch, p.B), p.lambdas, sketch="srht", m=1024,
                                seed=3, tol=1e-7, timing=1)
    X, rep = ctx.solve_path(dev(torch, p.A), dev(torch, p.B), p.lambdas, sketch="srht", m=1024,
                            seed=3, tol=1e-7, basis_prec=2, f32_switch=switch, timing=1)
    e64 = direct.rel_err(X64.cpu().numpy(), ref)
    err = direct.rel_err(X.cpu().numpy(), ref)
    print(f"mixed: max rel err {err.max():.3e} (FP64 path {e64.max():.3e}), "
          f"launches f32 {rep['ata_f32_launches']} f64 {rep['ata_launches']}, "
          f"k_sum {rep['k_sum']} vs {rep64['k_sum']}")
    assert rep["ata_f32_launches"] > 0 and rep["ata_launches"] > 0
    assert err.max() <= 1e-6, err


def test_fp64_matrix_ignores_fp32_request(torch, ctx):
    # FP64 storage: the products stay FP64 whatever basis_prec asks
    A = W.dense_decay(3000, 80, seed=4)
    B, _ = W.rhs(A, 1, 0.1, seed=5)
    lams = W.lambda_grid(1e-3, 1e2, 11)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch="srht", m=200, seed=1,
                            basis_prec=1, timing=1)
    assert rep["ata_f32_launches"] == 0
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(A, B, lams))
    assert err.max() <= 1e-6
