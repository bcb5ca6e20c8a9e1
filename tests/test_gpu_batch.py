"""Many small problems in one build (ihsbin_path_build_batch): every
problem's path matches the oracle's direct solve at every lambda, the paths
are independent handles, and the batch runs its steps once for all problems."""
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


def stack(torch, P, n, d, K, seed, dtype=np.float64):
    As, Bs = [], []
    for p in range(P):
        A = W.dense_decay(n, d, seed=seed + 2 * p, dtype=dtype)
        B, _ = W.rhs(A, K, 0.1, seed=seed + 2 * p + 1)
        As.append(A)
        Bs.append(B)
    dev = torch.device("cuda", 0)
    return As, Bs, torch.from_numpy(np.stack(As)).to(dev), torch.from_numpy(np.stack(Bs)).to(dev)


@pytest.mark.parametrize("kind,K,dt", [("gaussian", 1, np.float64), ("gaussian", 2, np.float32),
                                       ("srht", 1, np.float32), ("countsketch", 3, np.float64)])
def test_batch_paths_match_oracle(torch, ctx, kind, K, dt):
    P, n, d = 7, 2048, 96
    As, Bs, At, Bt = stack(torch, P, n, d, K, seed=300 + K, dtype=dt)
    lams = W.lambda_grid(1e-3, 1e2, 40)
    paths, rep = ctx.path_build_batch(At, Bt, 1e-3, 1e2, sketch=kind, m=64, seed=11, tol=1e-8)
    assert rep["status"] == 0 and len(paths) == P, rep
    for p in range(P):
        X = paths[p].eval(lams).cpu().numpy()
        err = direct.rel_err(X, direct.ridge_path(As[p], Bs[p], lams))
        assert err.max() <= 1e-6, (p, err.max())
    # handles are independent: freeing some leaves the others usable
    for p in range(0, P, 2):
        paths[p].free()
    X = paths[1].eval(lams[:5]).cpu().numpy()
    assert direct.rel_err(X, direct.ridge_path(As[1], Bs[1], lams[:5])).max() <= 1e-6
    for p in range(1, P, 2):
        paths[p].free()


@pytest.mark.parametrize("prec", [1, 2])
def test_batch_low_precision_gaussian_sketch(torch, ctx, prec):
    # BF16 (1) and FP8 (2) Gaussian sketches in a batched build: each problem
    # sketched on the matrix cores, every path within the bar
    P, n, d = 4, 2048, 96
    As, Bs, At, Bt = stack(torch, P, n, d, 1, seed=610 + prec, dtype=np.float32)
    lams = W.lambda_grid(1e-3, 1e2, 30)
    paths, rep = ctx.path_build_batch(At, Bt, 1e-3, 1e2, sketch="gaussian", m=64, seed=11,
                                      tol=1e-8, sketch_prec=prec)
    assert rep["status"] == 0 and len(paths) == P, rep
    for p in range(P):
        err = direct.rel_err(paths[p].eval(lams).cpu().numpy(),
                             direct.ridge_path(As[p], Bs[p], lams))
        assert err.max() <= 1e-6, (p, err.max())
        paths[p].free()


def test_batch_strided_and_noalloc_eval(torch, ctx):
    # problems taken every other block of a larger allocation (strides wider
    # than one problem), evaluated through the allocation-free entry point
    P, n, d = 5, 1500, 64
    As, Bs, At, Bt = stack(torch, 2 * P, n, d, 1, seed=900)
    paths, rep = ctx.path_build_batch(At[::2], Bt[::2], 1e-2, 1e1, sketch="gaussian", m=128, seed=3)
    lams = W.lambda_grid(1e-2, 1e1, 25)
    for p in range(P):
        out = torch.empty((len(lams), d, 1), dtype=torch.float64, device="cuda:0")
        paths[p].eval_noalloc(lams, out)
        assert torch.equal(out, paths[p].eval(lams))
        err = direct.rel_err(out.cpu().numpy(), direct.ridge_path(As[2 * p], Bs[2 * p], lams))
        assert err.max() <= 1e-6
        paths[p].free()


def test_batch_of_one_matches_oracle_and_rejects_csr(torch, ctx):
    from paper_2210_12212_amd import IhsbinError
    As, Bs, At, Bt = stack(torch, 1, 3000, 120, 2, seed=77, dtype=np.float32)
    paths, rep = ctx.path_build_batch(At, Bt, 1e-3, 1e2, sketch="srht", m=400, seed=5)
    lams = W.lambda_grid(1e-3, 1e2, 30)
    err = direct.rel_err(paths[0].eval(lams).cpu().numpy(), direct.ridge_path(As[0], Bs[0], lams))
    assert err.max() <= 1e-6
    paths[0].free()
    with pytest.raises(IhsbinError) as e:
        ctx.path_build_batch(At, Bt, 1e-3, 1e2, adaptive_m=2)
    assert e.value.status == -7


@pytest.mark.parametrize("graph_steps", [1, 3, 5])
def test_batch_basis_steps_in_hip_graphs(torch, ctx, graph_steps):
    # the basis steps captured into HIP graphs a few at a time give paths of
    # the same accuracy (the stop test runs once per graph, so the step count
    # can only grow)
    P, n, d = 6, 2048, 128
    As, Bs, At, Bt = stack(torch, P, n, d, 2, seed=500, dtype=np.float32)
    lams = W.lambda_grid(1e-3, 1e2, 30)
    p0, r0 = ctx.path_build_batch(At, Bt, 1e-3, 1e2, sketch="gaussian", m=128, seed=2)
    pg, rg = ctx.path_build_batch(At, Bt, 1e-3, 1e2, sketch="gaussian", m=128, seed=2,
                                  graph_steps=graph_steps)
    assert rg["status"] == 0 and rg["k_max_used"] >= r0["k_max_used"]
    assert rg["k_max_used"] <= r0["k_max_used"] + graph_steps - 1
    for p in range(P):
        X = pg[p].eval(lams).cpu().numpy()
        err = direct.rel_err(X, direct.ridge_path(As[p], Bs[p], lams))
        assert err.max() <= 1e-6, (p, err.max())
        if rg["k_max_used"] == r0["k_max_used"]:
            # same steps in the same order: the same bits
            assert torch.equal(pg[p].eval(lams), p0[p].eval(lams))
        pg[p].free()
        p0[p].free()
